/*
 * sharp.h -- C ABI of the MI355X (gfx950) RAAR ptychography hot path.
 *
 * Implements the data-parallel core of the SHARP solver (Marchesini et al.,
 * "SHARP: a distributed, GPU-based ptychographic solver", arXiv:1602.01448):
 * frames z_i = w . T_i psi (Sec. "Forward model", Eq. (overlap)), the unitary
 * 2-D DFT F with the e^{+2 pi i q.r} sign (Sec. "Forward model"), the data
 * projector P_a z = F*(Fz/|Fz|) a (Eq. (Pa)), the overlap projector
 * P_Q = Q (Q*Q)^{-1} Q* (Eq. (Pq)), the RAAR update of the algorithm box
 * (step 5), the object update psi = Q*z/Q*Q (Eq. (standardobject)) and the
 * probe update (Eq. (standardprobe)).
 *
 * Conventions for every call:
 *  - Complex arrays are interleaved complex64 (re, im float pairs), row-major,
 *    y-major.  Frame stacks are [K][m][m]; objects are [ny][nx]; probes [m][m].
 *  - Diffraction data are float32 [K][m][m] intensities with the zero
 *    frequency at index [0][0] (no fftshift), in the F convention above.
 *  - Positions are int32 [K][2] top-left frame corners (y, x) in object
 *    pixels (Sec. "Forward model": x_i on the integer grid 0..n-m).
 *  - Pointers named d_* are device pointers (caller-owned, on the current
 *    HIP device); pointers named h_* are host pointers.  The library never
 *    allocates or frees device memory: all its device state lives in one
 *    caller-provided workspace (sharp_workspace_bytes / sharp_set_workspace).
 *  - Every device call is enqueued asynchronously on the plan's stream
 *    (sharp_set_stream; default: the null stream).  Only sharp_get_metrics,
 *    sharp_sync and sharp_grad's loss read-back (none) synchronise.
 *  - Every call returns SHARP_OK (0) or a negative status; no exception or
 *    abort crosses the ABI.  A plan is not thread-safe; distinct plans are
 *    independent.
 */
#ifndef SHARP_H
#define SHARP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sharp_plan_s* sharp_plan;
typedef struct sharp_batch_s* sharp_batch;

enum sharp_status {
    SHARP_OK = 0,
    SHARP_ERR_INVALID_ARG = -1,           /* null pointer, bad count, beta outside (0,1] */
    SHARP_ERR_UNSUPPORTED_SIZE = -2,      /* m not in {16,32,64,128,256}, m > n */
    SHARP_ERR_POSITION_OUT_OF_RANGE = -3, /* a frame leaves the object (non-periodic) */
    SHARP_ERR_NOT_READY = -4,             /* workspace / data / probe / object missing */
    SHARP_ERR_WORKSPACE_TOO_SMALL = -5,
    SHARP_ERR_NONFINITE = -6,             /* NaN/Inf seen in data or in an iterate */
    SHARP_ERR_HIP = -7,                   /* a HIP runtime call failed */
    SHARP_ERR_HOST_ALLOC = -8,            /* host metadata allocation failed */
    SHARP_ERR_SCRATCH_LIMIT = -9          /* sharp_apply_noalloc: the operator needs more scratch
                                             than SHARP_NOALLOC_SCRATCH_BYTES */
};

/* Static text for a status code (never NULL). */
const char* sharp_status_string(int status);

/* Options of a plan (user options of Sec. "Computational Methodology":
 * probe-retrieval frequency, plus the boundary mode used by the paper's
 * benchmark, Fig. "timing" caption).  Zero-initialised = defaults. */
typedef struct sharp_options {
    int periodic;     /* 0: frames lie inside the object, 0 <= y <= ny-m, 0 <= x <= nx-m;
                         1: frames wrap modulo (ny, nx); positions in [0,ny) x [0,nx) */
    int probe_every;  /* 0: probe is known; k > 0: probe update every k iterations */
    int probe_start;  /* first iteration (1-based, counted over the plan's life) with a
                         probe update; 0 means 1 */
    float eps_D;      /* (Q*Q)^{-1} is 1/D where D > eps_D and 0 elsewhere (default 0) */
    int tile;         /* merge tile side in object pixels: 16, 32 or 64 (0 = the library's
                         choice: 32 while that gives >= 1024 tiles, else 16) */
    int merge_split;  /* frame chunks per tile in the first pass of the tile merges (RAAR,
                         object output, density, gradient), >= 1 (0 = the library's choice:
                         >= 1024 workgroups, >= 4 frames per chunk) */
    int grad_groups;  /* workgroups of the gradient frame kernel (0 = the library's choice).
                         The Python binding's Plan.tuned fills these from the autotuner's
                         cache for the geometry. */
    int frame_launch; /* m = 128: 0 or 2 = carry kept in the Fourier domain (default),
                         1 = carry in frame space (3 is taken as 2).  m = 256 RAAR:
                         0 = default (3 when K >= 400, else 2; 1 when the object is
                         wider than 8192); 1 = row, column and row passes with the carry
                         in frame space, then the tile merge; 2 = carry kept in the
                         Fourier domain, a column pass reading the row-transformed
                         gather that the previous strip merge prepared; 3 = carry in
                         the Fourier domain, the column pass (a quarter of a frame's
                         columns per workgroup) forms its own row transform and the
                         strip merge only merges.  m < 128: ignored (frame space).
                         Values outside 0..3 are rejected */
    int fft_block;    /* m = 256, form 1: threads per pass workgroup, 128, 256 or 512 (8, 16
                         or 32 rows / columns per workgroup); 0 = 256 */
    int strip_rows;   /* m = 256, forms 2 and 3: object rows per merge strip, 1 or 2 (0 =
                         default, 1); 2 is taken only while 2 nx <= 8192 */
    int probe_center; /* 1: after every probe update, roll the probe circularly by the integer
                         that brings the centroid of |w|^2 within half a pixel of (m/2, m/2)
                         (algorithm box, step 7, centre-of-mass drift correction); 0: off */
    int reserved[1];  /* must be zero */
} sharp_options;

/* ------------------------------------------------------------------------
 * Plan: geometry (Sec. "Forward model") and host-side set-up (algorithm box,
 * step 4: build Q, Q*, (Q*Q)^{-1}).  Host only; touches no device.
 *   nx, ny   object size, 1 <= m <= min(nx, ny)
 *   m        frame side, one of 16, 32, 64, 128, 256
 *   K        number of frames, >= 1
 *   h_pos_yx host int32 [K][2], copied
 *   opt      NULL = defaults
 * Errors: INVALID_ARG, UNSUPPORTED_SIZE, POSITION_OUT_OF_RANGE, HOST_ALLOC.
 * ---------------------------------------------------------------------- */
int sharp_plan_create(sharp_plan* out, int nx, int ny, int m, int K,
                      const int32_t* h_pos_yx, const sharp_options* opt);
void sharp_plan_destroy(sharp_plan plan);

/* Bytes of device workspace the plan needs (256-byte aligned start). */
size_t sharp_workspace_bytes(sharp_plan plan);
/* Attach the workspace (caller-owned device memory, >= sharp_workspace_bytes)
 * and upload the plan's tables into it.  Resets data/probe/object state.
 * Errors: INVALID_ARG (null / misaligned), WORKSPACE_TOO_SMALL, HIP. */
int sharp_set_workspace(sharp_plan plan, void* d_workspace, size_t bytes);
/* Stream (a hipStream_t) that every later call enqueues on; NULL = null stream. */
int sharp_set_stream(sharp_plan plan, void* stream);

/* ------------------------------------------------------------------------
 * Inputs (algorithm box, step 1)
 * ---------------------------------------------------------------------- */
/* Measured intensities d_I float32 [K][m][m].  Stores the variance-stabilised
 * amplitudes a = sqrt(max(I, 0)) (Sec. "Forward model") and ||a||.  d_I is
 * read only.  NaN/Inf inputs are reported as NONFINITE by the next
 * sharp_get_metrics / sharp_sync. */
int sharp_set_data(sharp_plan plan, const float* d_I);
/* Probe w, complex64 [m][m] (copied).  Rebuilds D = diag(Q*Q) (Eq. (Pq)). */
int sharp_set_probe(sharp_plan plan, const void* d_w);
/* Initial probe from the data (algorithm box, step 2): w0 = F^{-1} sqrt of
 * the mean frame, shifted by (m/2, m/2) to the frame centre.  Needs data. */
int sharp_init_probe(sharp_plan plan);
/* Constraint on every probe update (algorithm box, step 7; Sec. "Phase
 * retrieval", Fourier-space drifts):
 *   kind 0: none (default);
 *   kind 1: Fourier mask m_w:       w := F^{-1}{ (F w) m_w };
 *   kind 2: Fourier amplitudes a_w: w := F^{-1}{ sgn(F w) a_w }, sgn(0) := 1.
 * F is the frame transform of the data (unitary, DC at [0][0]).  d_values:
 * float32 [m][m] device pointer, copied into the workspace (ignored and may
 * be NULL for kind 0).  It is applied before the centre-of-mass correction
 * (option probe_center).  Not part of the checkpoint state.
 * Errors: INVALID_ARG (kind outside 0..2, NULL values), NOT_READY (no
 * workspace), HIP. */
int sharp_set_probe_constraint(sharp_plan plan, int kind, const float* d_values);
/* Start image psi0, complex64 [ny][nx] (copied); sets z^(0) = Q psi0
 * (algorithm box, step 4) and restarts the iteration counter.  Needs probe. */
int sharp_set_object(sharp_plan plan, const void* d_psi);

/* ------------------------------------------------------------------------
 * Iterate (algorithm box, steps 5-7)
 * n iterations of z <- [2b P_Q P_a + (1-2b) P_a + b (I - P_Q)] z, beta in
 * (0, 1] (the paper recommends (0.5, 1], default 0.75).  The sign of the last
 * term is the relaxed-averaged-alternating-reflections one; the sign printed
 * in the algorithm box diverges.  With probe_every > 0 the probe is updated
 * by Eq. (standardprobe) after the object update of due iterations.  eps_a
 * of the z entering each iteration is recorded on the device.
 * Errors: INVALID_ARG, NOT_READY (no data, probe or object), HIP.
 * ---------------------------------------------------------------------- */
int sharp_raar_iterate(sharp_plan plan, int n, float beta);

/* ------------------------------------------------------------------------
 * Outputs (algorithm box, steps 6 and 9)
 * ---------------------------------------------------------------------- */
/* psi^(l) = Q* z^(l) / Q*Q (Eq. (standardobject)), 0 where no frame
 * illuminates; complex64 [ny][nx]. */
int sharp_get_object(sharp_plan plan, void* d_psi_out);
/* Current probe w, complex64 [m][m]. */
int sharp_get_probe(sharp_plan plan, void* d_w_out);
/* Synchronises the stream.  Copies up to max_n recorded eps_a values
 * (Eq. (amplitudemetric)), oldest first, of the iterations since the last
 * sharp_set_object, into h_eps_a; *n_written gets the count.  The history
 * keeps the last 4096 values.  Returns NONFINITE if a non-finite value was
 * seen in the data or an iterate. */
int sharp_get_metrics(sharp_plan plan, float* h_eps_a, int max_n, int* n_written);
/* Synchronises the plan's stream and reports the non-finite flag. */
int sharp_sync(sharp_plan plan);

/* ------------------------------------------------------------------------
 * Amplitude loss and gradient (Eq. (data0) as a least-squares loss)
 * L(psi, w) = sum_i sum_q (|F(w . T_i psi)|_q - a_iq)^2 with the plan's data,
 * and its gradient in the complex convention g = dL/dRe + i dL/dIm:
 *   g_psi = Q* r,  g_w = sum_i conj(T_i psi) r_i,  r = 2 (z - P_a z),  z = Q_w psi.
 * d_psi complex64 [ny][nx], d_w complex64 [m][m] (inputs, read only);
 * d_loss float32 [1], d_gpsi complex64 [ny][nx], d_gw complex64 [m][m]
 * (outputs; d_gpsi or d_gw may be NULL to skip).  Needs data.  Does not
 * touch the RAAR state except scratch.
 * ---------------------------------------------------------------------- */
int sharp_grad(sharp_plan plan, const void* d_psi, const void* d_w,
               float* d_loss, void* d_gpsi, void* d_gw);

/* Forward model I_i = |F(w . T_i psi)|^2 (Eq. (data0)) into d_I_out float32
 * [K][m][m]; used to synthesise data.  d_psi [ny][nx], d_w [m][m]. */
int sharp_simulate(sharp_plan plan, const void* d_psi, const void* d_w, float* d_I_out);

/* ------------------------------------------------------------------------
 * Individual operators of the method, on caller buffers, with the plan's
 * current probe (and data for SHARP_OP_PA).  Used to check each projection.
 *   SHARP_OP_F      frames -> F frames              (Sec. "Forward model")
 *   SHARP_OP_FINV   frames -> F* frames
 *   SHARP_OP_Q      object -> w . T_i object        (Eq. (overlap))
 *   SHARP_OP_QSTAR  frames -> sum_i T_i^T conj(w) z_i
 *   SHARP_OP_PA     frames -> P_a frames            (Eq. (Pa))
 *   SHARP_OP_PQ     frames -> Q (Q*Q)^+ Q* frames   (Eq. (Pq))
 *   SHARP_OP_OBJECT frames -> (Q*Q)^+ Q* frames     (Eq. (standardobject))
 * "frames" are complex64 [K][m][m]; "object" complex64 [ny][nx].  d_in and
 * d_out must not overlap.  Needs probe (and data for PA).
 * ---------------------------------------------------------------------- */
enum sharp_op {
    SHARP_OP_F = 0, SHARP_OP_FINV = 1, SHARP_OP_Q = 2, SHARP_OP_QSTAR = 3,
    SHARP_OP_PA = 4, SHARP_OP_PQ = 5, SHARP_OP_OBJECT = 6
};
int sharp_apply(sharp_plan plan, int op, const void* d_in, void* d_out);

/* ------------------------------------------------------------------------
 * For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * operators as sharp_apply, same arguments and results, with their scratch
 * taken from a fixed array of SHARP_NOALLOC_SCRATCH_BYTES that the library
 * holds on each device it runs on (from the first call on that device until
 * the process ends) instead of from the plan's workspace.  The scratch is
 * the m = 256 stage buffer of F, F* and P_a (K m^2 complex64), the residual
 * partials of P_a, the object temporary of P_Q (ny nx complex64) and the
 * frame-chunk partials of a split merge.  Allocates and frees nothing.
 * Every call on one device shares that device's array: calls that overlap
 * on one device (several streams or host threads) race.  Must be called with
 * the plan's device current.
 * Errors: as sharp_apply, and SCRATCH_LIMIT (checked first, before any
 * device work) when the operator needs more scratch than the array holds.
 * ---------------------------------------------------------------------- */
#define SHARP_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int sharp_apply_noalloc(sharp_plan plan, int op, const void* d_in, void* d_out);

/* ------------------------------------------------------------------------
 * Checkpoint / resume of the iteration state (carry frames, object terms,
 * probes, counters).  d_state is a device buffer of sharp_state_bytes(plan)
 * bytes laid out as consecutive segments, each starting on a 256-byte
 * boundary: carry u complex64 [K][m][m] (z^(l) = u + g w_g T psi_v), psi_v
 * complex64 [ny][nx], psi^(l) of the last probe-update iteration complex64
 * [ny][nx], current probe w complex64 [m][m], carry probe w_g complex64
 * [m][m], eps_a history float32 [4096], then a small header.  set_state
 * needs data to have been set; it rebuilds D from the restored probe.  It
 * returns INVALID_ARG, before touching the plan, for a header of another
 * geometry or with out-of-range fields (negative counters, a gather
 * coefficient outside [0, 1] or not finite, flags other than 0 or 1).
 * ---------------------------------------------------------------------- */
size_t sharp_state_bytes(sharp_plan plan);
int sharp_get_state(sharp_plan plan, void* d_state);
int sharp_set_state(sharp_plan plan, const void* d_state);

/* ------------------------------------------------------------------------
 * Host-side introspection (no device work).
 * ---------------------------------------------------------------------- */
typedef struct sharp_plan_info {
    int nx, ny, m, K, periodic;
    int tile, tiles_x, tiles_y, merge_split, grad_groups, frame_launch, fft_block;
    int strip_rows;           /* form 2: object rows per merge strip (0 in form 1) */
    int streaming;            /* 1: the frame arrays (K m^2 complex values) exceed the GPU's 256 MiB
                                 last-level cache and the frame passes use streaming (nontemporal)
                                 loads and stores for them; 0: cached accesses */
    long long csr_nnz;        /* (tile, frame) incidences */
    long long iteration;      /* iterations run since sharp_set_object */
} sharp_plan_info;
int sharp_get_plan_info(sharp_plan plan, sharp_plan_info* info);
/* CSR of tiles -> frames (frames ascending in each tile, tiles row-major):
 * h_ptr int32 [tiles+1], h_frames int32 [csr_nnz]. */
int sharp_get_plan_csr(sharp_plan plan, int32_t* h_ptr, int32_t* h_frames);

/* ------------------------------------------------------------------------
 * Kernel timing (diagnostics).  While enabled, the launches of
 * sharp_raar_iterate and sharp_grad are bracketed by HIP events on the
 * plan's stream, per category: 0 frame kernel (m <= 128: the whole fused
 * kernel; m = 256: the row pass with the gather), 1 column pass (m = 256),
 * 2 output row pass (m = 256), 3 merge, 4 residual reduction, 5 probe
 * update, 6 copies.  sharp_timing_read synchronises, adds the elapsed
 * milliseconds and launch counts of the finished pairs into h_ms[8] and
 * h_launches[8] (overwritten) and forgets them.
 * ---------------------------------------------------------------------- */
int sharp_timing_enable(sharp_plan plan, int on);
int sharp_timing_read(sharp_plan plan, double* h_ms, long long* h_launches);

/* ------------------------------------------------------------------------
 * Batched execution of independent plans (one launch sequence per
 * iteration, all scans together).  Each plan keeps its own state and must
 * have data, probe and object set; the plans' streams are ignored and the
 * batch's stream is used.  Plans with probe_every > 0 are rejected.
 * The plans must outlive the batch.  sharp_batch_set_workspace records the
 * workspace each plan has at that moment (its device pointers go into the
 * batch's launch arguments): if a plan is given another workspace later
 * (sharp_set_workspace), sharp_batch_raar_iterate returns NOT_READY before
 * any launch until sharp_batch_set_workspace is called again.
 * ---------------------------------------------------------------------- */
int sharp_batch_create(sharp_batch* out, int nplans, const sharp_plan* plans);
void sharp_batch_destroy(sharp_batch batch);
size_t sharp_batch_workspace_bytes(sharp_batch batch);
int sharp_batch_set_workspace(sharp_batch batch, void* d_workspace, size_t bytes);
int sharp_batch_set_stream(sharp_batch batch, void* stream);
int sharp_batch_raar_iterate(sharp_batch batch, int n, float beta);

/* ------------------------------------------------------------------------
 * Device read-rate reference (a measurement utility, not part of the method;
 * for benchmarks that compare the passes above with what the GPU's memory
 * delivers): reads `bytes` bytes from d_src with 16-byte nontemporal loads,
 * eight requests in flight per thread, SHARP_READ_REFERENCE_SINK workgroups
 * of 256 threads striding over the buffer, and writes one float per
 * workgroup to d_sink (SHARP_READ_REFERENCE_SINK floats, device memory; the
 * values carry no meaning).  Asynchronous on `stream` (a hipStream_t; NULL =
 * null stream).  d_src must be 16-byte aligned and bytes a positive multiple
 * of 16, else SHARP_ERR_INVALID_ARG; a failed launch gives SHARP_ERR_HIP.
 * ---------------------------------------------------------------------- */
#define SHARP_READ_REFERENCE_SINK 2048
int sharp_read_reference(const void* d_src, size_t bytes, float* d_sink, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SHARP_H */
