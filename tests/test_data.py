"""The synthetic scan recipes: sizes, frame counts, position ranges and
reproducibility of the seeded streams."""
import numpy as np
import pytest

from sharp_data import gen


@pytest.mark.parametrize("cfg,n,m,K", [(1, 128, 32, 169), (2, 512, 64, 841), (3, 2048, 256, 2025),
                                       (4, 512, 128, 1024), ("4s", 64, 16, 25)])
def test_config_shapes(cfg, n, m, K):
    s = gen.config_scan(cfg)
    assert (s.n, s.m, s.K) == (n, m, K)
    assert s.positions.dtype == np.int32 and s.positions.shape == (K, 2)
    assert s.positions.min() >= 0 and s.positions.max() <= n - m
    assert s.obj.shape == (n, n) and s.probe.shape == (m, m) and s.psi0.shape == (n, n)
    assert np.all(s.psi0.imag == 0) and s.psi0.real.min() >= 0 and s.psi0.real.max() < 1


def test_reproducible():
    a, b = gen.config_scan(2), gen.config_scan(2)
    assert np.array_equal(a.positions, b.positions) and np.array_equal(a.obj, b.obj)
    assert np.array_equal(a.psi0, b.psi0)


def test_recipes():
    s1 = gen.config_scan(1)
    amp = np.abs(s1.obj)
    assert amp.min() >= 0.5 and amp.max() <= 1.0
    assert np.abs(np.angle(s1.obj)).max() <= np.pi / 2
    assert np.array_equal(s1.positions[:3], [[0, 0], [0, 8], [0, 16]])
    s2 = gen.config_scan(2)
    assert np.allclose(np.abs(s2.obj), 1.0)
    r2 = (np.arange(64)[:, None] - 32) ** 2 + (np.arange(64)[None, :] - 32) ** 2
    assert np.all(s2.probe[r2 > 400] == 0) and np.all(np.abs(s2.probe[r2 <= 400]) > 0.999)
    d = s2.positions - np.array([(16 * j, 16 * k) for j in range(29) for k in range(29)])
    assert np.abs(d).max() <= 2


def test_poisson_scaling():
    rng = np.random.default_rng(0)
    I = rng.uniform(0, 1, (50, 8, 8))
    out, c = gen.apply_poisson(I, 1e6, np.random.default_rng(1))
    assert out.dtype == np.float32
    assert abs(out.sum() / 50 / 1e6 - 1) < 1e-3
    assert abs(c - 1e6 / (I.sum() / 50)) < 1e-6 * c


def test_batch_scans():
    scans = gen.batch_scans()
    assert len(scans) == 32
    for s in scans:
        assert 256 <= s.n <= 1024 and s.m in (64, 128, 256) and s.m <= s.n // 2
        assert 100 <= s.K <= 1500
        assert s.positions.min() >= 0 and s.positions.max() <= s.n - s.m
    assert len({s.m for s in scans}) == 3


def test_shard_share_partitions_the_frames():
    """The strip shares of the large-frame scan partition its frames; each
    share's positions fit its strip + halo, and its object rows are the
    scan's rows from the strip start."""
    s = gen.config_scan(3)
    seen = []
    for g in range(8):
        sh = gen.shard_share(s, g, 8)
        pos = sh["positions"]
        assert 200 <= len(pos) <= 320   # about K / 8 each
        assert pos[:, 0].min() >= 0 and pos[:, 0].max() < (s.n - s.m + 1 + 7) // 8
        assert (pos[:, 0] + s.m <= sh["ny"]).all() and (pos[:, 1] + s.m <= sh["nx"]).all()
        assert np.array_equal(pos[:, 0] + sh["row0"], s.positions[sh["frames"], 0])
        assert np.array_equal(sh["obj"], s.obj[sh["row0"]:sh["row0"] + sh["ny"]])
        seen.extend(sh["frames"].tolist())
    assert sorted(seen) == list(range(s.K))
