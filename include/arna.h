/*
 * arna.h -- C interface of the MI355X (gfx950) particle-filter step with
 * RNA / ARNA distributed resampling.
 *
 * Method: Demirel, Smal, Niessen, Meijering, Sbalzarini, "An Adaptive
 * Distributed Resampling Algorithm with Non-Proportional Allocation"
 * (arXiv:1310.4624).  One call of pf_step is one iteration of Alg. 3 (ARNA)
 * or Alg. 2 (RNA): ring, exchange ratio, particle exchange, renormalization,
 * (P) and (U) of Alg. 1, per-PE estimate and weight, local systematic
 * resampling, weight reset, master estimate.  A processing element (PE) is
 * one GPU workgroup that owns a fixed block of N_p particles (Sec. III-A).
 *
 * Conventions for every entry point:
 *   - Return value: PF_OK (0) or a negative PF_E* code; nothing throws across
 *     this interface.  pf_strerror() gives the text.
 *   - "device" pointers are HIP device memory (e.g. torch CUDA tensors on
 *     ROCm); "host" pointers are ordinary CPU memory.  The caller owns every
 *     pointer it passes; the library owns all particle buffers.
 *   - Work is enqueued on pf_config.stream (NULL = the default stream).  Only
 *     pf_estimate, pf_debug_* and pf_destroy synchronize with the host.
 *   - Particle state is float32 and component-major: [5][N] for
 *     (x, y, vx, vy, I), N = n_filters * n_pe * n_per_pe; slot (f, m, s) is
 *     column ((f * n_pe) + m) * n_per_pe + s.  x is the image column, y the
 *     row; pixel (u, v) has its centre at (u, v).
 */
#ifndef ARNA_H
#define ARNA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    PF_OK = 0,
    PF_EINVAL = -1,        /* bad argument or configuration */
    PF_ENOMEM = -2,        /* device allocation failed */
    PF_EHIP = -3,          /* a HIP runtime call failed */
    PF_ENUMERIC = -4,      /* a log-weight was NaN (e.g. a NaN pixel); sticky */
    PF_ESTATE = -5,        /* call out of order (e.g. pf_exchange twice) */
    PF_EUNSUPPORTED = -6,  /* size beyond the limits below */
    PF_ETIMEOUT = -7       /* workgroups of a multi-iteration launch waited for each
                              other longer than 2 s (results undefined); sticky */
};

enum { PF_MODE_RNA = 0, PF_MODE_ARNA = 1 };
enum { PF_INIT_TRACKING = 0, PF_INIT_INFOSHARE = 1 };
enum { PF_LIK_PATCH = 0, PF_LIK_POINT = 1, PF_LIK_POISSON = 2 };
/* How pf_run launches its iterations (pf_config.launch). */
enum { PF_LAUNCH_AUTO = 0,        /* the library's choice: currently one launch per
                                     iteration (see pf_config.launch) */
       PF_LAUNCH_STEPWISE = 1,    /* one launch per iteration */
       PF_LAUNCH_PERSISTENT = 2   /* multi-iteration launches; pf_init fails with
                                     PF_EUNSUPPORTED when the context cannot use them */ };

/* Debug flags (pf_config.debug). */
enum { PF_DEBUG_TRACE = 1,    /* keep Q, ancestors, propagated state, ... of the last step */
       PF_DEBUG_LINEAGE = 2   /* carry an int32 lineage tag per particle */ };

/* Limits of this build. */
#define PF_MAX_PE 8192u
#define PF_MAX_PER_PE 65536u
/* Up to this many particles per PE a PE's particles live in LDS for the whole
 * iteration.  Larger PEs stream them through HBM (other step kernels with the
 * same results up to the summation order of the FP64 PE sums; with fewer than
 * 256 PEs each PE is split over several workgroups): such contexts take no
 * block_size other than 0 or 1024, no pes_per_wg above 1 (PF_EINVAL), no
 * PF_DEBUG_LINEAGE, no PF_LAUNCH_PERSISTENT and no gradient recording
 * (PF_EUNSUPPORTED), and hold N more floats of device
 * memory (the log-weights of the iteration). */
#define PF_MAX_PER_PE_LDS 4096u
#define PF_MAX_PATCH 15u
#define PF_MAX_PARTICLES (1u << 29)   /* F M N_p: state indices are 32-bit (5 F M N_p < 2^32) */

typedef struct pf_ctx pf_ctx;   /* opaque; created by pf_init, freed by pf_destroy */

typedef struct {
    uint32_t struct_size;       /* = sizeof(pf_config); ABI check */
    uint32_t n_filters;         /* F: independent filters (one tracked object each);
                                   F M <= 2^24 and F M N_p <= PF_MAX_PARTICLES */
    uint32_t n_pe;              /* M: PEs per filter, 1..PF_MAX_PE */
    uint32_t n_per_pe;          /* N_p: particles per PE, 1..PF_MAX_PER_PE */
    uint32_t width, height;     /* frame size in pixels (patch mode) */
    uint32_t patch;             /* odd patch side, 1..PF_MAX_PATCH (9 in the benchmarks) */
    uint32_t mode;              /* PF_MODE_RNA: fixed ring, N_ex = floor(fixed_ratio N_p)
                                   PF_MODE_ARNA: random ring (Sec. IV-B), N_ex by Eq. 3 */
    uint32_t init_mode;         /* PF_INIT_TRACKING or PF_INIT_INFOSHARE (Sec. V) */
    uint32_t lik_mode;          /* PF_LIK_PATCH (image, Gaussian pixel noise),
                                 * PF_LIK_POINT (position data) or PF_LIK_POISSON
                                 * (image of photon counts: Poisson pixel noise around
                                 * B + I g, the noise of the paper's Fig. 1; needs B > 0) */
    float fixed_ratio;          /* RNA exchange ratio N_ex/N_p, in [0, 1] */
    float initial_ratio;        /* ARNA ratio of the first iteration, in [0, 1] */
    float eff_cutoff;           /* ARNA: no exchange when PE_eff > eff_cutoff * M;
                                   values outside (0, 1) disable the cut-off */
    float psf_sigma;            /* spot profile width (px), > 0 */
    float background;           /* image background level */
    float noise_sigma;          /* pixel noise std (patch) or position noise std (point), > 0 */
    float q;                    /* NCV process-noise intensity (px^2), >= 0 */
    float sigma_I;              /* intensity random-walk std, >= 0 */
    uint32_t debug;             /* PF_DEBUG_* flags */
    uint32_t ring_groups;       /* ARNA ring: 0 or 1 = one random ring over all PEs
                                 * (Sec. IV-B); G in 2..256 = hardware-aware ring (the
                                 * future work of Sec. VI): PE m of filter f is in group
                                 * (f M + m) mod G -- with G = 8 the MI355X die its
                                 * workgroup runs on -- and the ring visits the groups in
                                 * a random order and each group's PEs in a random order,
                                 * so only G of its M edges join different groups */
    uint32_t block_size;        /* threads per workgroup (one workgroup per PE): 0 = the
                                 * default (N_p rounded up to 64, at most 1024); else a
                                 * multiple of 64 in 64..1024 with block_size * P >= N_p
                                 * for P = 1, 2 or 4 slots per thread (the smallest such P
                                 * is used) -- the knob of the autotuner.  Above
                                 * PF_MAX_PER_PE_LDS particles per PE: 0 or 1024 */
    uint32_t launch;            /* PF_LAUNCH_*.  A multi-iteration launch runs up to 64
                                 * iterations with every PE's workgroup resident on its
                                 * compute unit: its resampled particles stay in registers,
                                 * only received slots are read back, and the PEs of a filter
                                 * meet at a barrier between iterations instead of a launch
                                 * boundary.  It needs a 9 x 9 patch or point data, no debug
                                 * flag, M < 2048 (else PF_EUNSUPPORTED), and F M
                                 * workgroups resident at once
                                 * (cooperative launch; e.g. F M <= 256 at N_p = 4096 on
                                 * MI355X).  Results are bitwise those of one launch per
                                 * iteration below 512 PEs (from 512 PEs on, one launch
                                 * per iteration is followed by the master step computed
                                 * once per filter, with another FP64 summation order;
                                 * a multi-iteration context keeps the order of its own
                                 * launches).  Iterations that record a gradient tape or
                                 * replay forced choices always run one launch each.  The
                                 * barrier costs less than a launch boundary only for small
                                 * contexts (about 10-15% faster up to 64 PEs), and the
                                 * cooperative launch it needs costs about 1 ms once the
                                 * process uses three or more other streams, so AUTO does
                                 * not choose it. */
    uint32_t pes_per_wg;        /* PEs per workgroup: 0 or 1 = one (k_step); P in 2..16 = P
                                 * PEs of one filter share a workgroup, each on its own
                                 * group of whole waves (block_size / P threads, a multiple
                                 * of 64, with block_size / P * 4 >= N_p; block_size 0 = P
                                 * times N_p rounded up to 64, at most 1024 / P): the PEs
                                 * share the image tile, the barriers and the launch's
                                 * workgroup count, which pays for small N_p.  Same
                                 * results as one PE per workgroup up to the summation
                                 * order of the FP64 PE sums.  N_p <= PF_MAX_PER_PE_LDS;
                                 * no PF_DEBUG_LINEAGE, no PF_LAUNCH_PERSISTENT
                                 * (PF_EUNSUPPORTED).  The autotuner's second axis. */
    uint64_t seed;              /* Philox key */
    void *stream;               /* hipStream_t or NULL */
} pf_config;

/* Host-side result of pf_estimate.  Arrays are caller-allocated; every
 * pointer except x_global may be NULL. */
typedef struct {
    double *x_global;           /* [F][5] master estimate x_k (Alg. 3, last step) */
    double *x_pe;               /* [F][M][5] per-PE estimates x^m_k */
    double *log_mass_pe;        /* [F][M] log W^(m)_k */
    double *log_mass_glob;      /* [F] log W_k = log sum_m W^(m)_k */
    double *pe_eff;             /* [F] PE_eff of iteration k (Eq. 4), in [1, M] */
    uint32_t *n_ex;             /* [F] N_ex used in iteration k */
    uint32_t *n_ex_next;        /* [F] N_ex that iteration k+1 will use */
    double *log_z_inc;          /* [F] log p(z_k | z_1:k-1), likelihood-ratio form */
    uint64_t step;              /* k: iterations completed */
} pf_estimate_t;

/* The master step of one iteration for one filter (Alg. 3, steps 9-10): what
 * the master computes from the PE records and broadcasts. */
typedef struct {
    double xhat[5];             /* x_k = sum_m W^(m)_k x^m_k / W_k */
    double log_mass_glob;       /* log W_k = log sum_m W^(m)_k */
    double pe_eff;              /* PE_eff of Eq. 4 on the integer PE masses
                                   P_m = floor(exp(L_m - max L) 2^20), in [1, M]; 0 without mass */
    double log_z_inc;           /* log p(z_k | z_1:k-1) in likelihood-ratio form: log W_k - log N_p */
    uint32_t n_ex;              /* N_ex used in iteration k */
    uint32_t n_ex_next;         /* N_ex iteration k+1 will use (Eq. 3; the fixed rules in RNA) */
    uint64_t step;              /* k */
} pf_master_t;

/* Per-PE record, the message each PE sends to the master (Alg. 3, step 9). */
typedef struct {
    double log_mass;            /* log W^(m)_k */
    double xhat[5];             /* x^m_k */
    float lstar;                /* max_i of the PE's log-weights */
    uint32_t total_q;           /* sum of the PE's fixed-point weights */
} pf_pe_record;

/* Create a filter context and initialize its particles (Sec. V: tracking or
 * information-sharing start).  truth: host [F][5] true initial states.
 * On success *out owns device memory until pf_destroy. */
int pf_init(const pf_config *cfg, const float *truth, pf_ctx **out);

/* One full iteration (Alg. 3 steps 1-10; Alg. 2 for RNA) on frame z_k.
 * d_frame: device float32, [height][width] row-major (patch mode) or
 * [F][2] observed positions (point mode).  Enqueue only: the frame must stay
 * valid until the stream has passed this step.  No host synchronization. */
int pf_step(pf_ctx *c, const float *d_frame);

/* n_steps iterations on consecutive frames d_frames + i * frame_stride
 * (stride in floats).  Same semantics as n_steps calls of pf_step. */
int pf_run(pf_ctx *c, const float *d_frames, uint32_t n_steps, uint64_t frame_stride);

/* pf_run that also writes the master step of every iteration (Alg. 3, steps
 * 9-10: global estimate, W_k, PE_eff, N_ex, likelihood increment) to
 * d_traj[i][f] (device, caller-owned, n_steps x F pf_master_t, 8-byte
 * aligned), so a tracker gets the estimate of every frame without a host
 * synchronization.  Iterations then run one launch each (never the
 * multi-iteration launch).  d_traj may be NULL (then this is pf_run).
 * Enqueue only. */
int pf_run_traj(pf_ctx *c, const float *d_frames, uint32_t n_steps, uint64_t frame_stride,
                pf_master_t *d_traj);

/* pf_run that also times every launch with a pair of HIP events recorded on
 * the context's stream around it, then synchronizes the stream.  host_ms_out
 * (host float [n_steps]) receives each iteration's duration in milliseconds:
 * that of its launch divided by the iterations the launch ran (the ring table
 * build of every 64th iteration included). */
int pf_run_timed(pf_ctx *c, const float *d_frames, uint32_t n_steps, uint64_t frame_stride,
                 float *host_ms_out);

/* *host_multi = 1 if pf_run may use multi-iteration launches for this context
 * (see pf_config.launch), else 0. */
int pf_run_info(const pf_ctx *c, uint32_t *host_multi);

/* Steps 1-3 of the next iteration alone (Alg. 3; Sec. III-A/C, IV-A/B):
 * ring, exchange ratio and particle exchange.  If d_src_map (device int64 [N])
 * is non-NULL it receives the composite source map: slot g is refilled from
 * slot d_src_map[g] of the previous iteration.  The next pf_step then performs
 * steps 4-10 with this exchange.  Calling it twice without a pf_step in
 * between returns PF_ESTATE. */
int pf_exchange(pf_ctx *c, int64_t *d_src_map);

/* Synchronize the stream and report the last completed iteration (master
 * estimate, W, PE_eff, N_ex, log-likelihood increment).  Returns PF_ENUMERIC
 * if any iteration so far produced a NaN log-weight (the flag is sticky). */
int pf_estimate(pf_ctx *c, pf_estimate_t *out);

/* -------------------------------------------------------------- batches */
/* Many independent filters advanced together: every iteration of
 * pf_batch_run issues one launch per group of contexts that share the kernel
 * variant (slots per thread, workgroup size, the 9 x 9 patch with Gaussian or
 * Poisson noise, or point data) instead of one launch per context; the work
 * of each workgroup is exactly that of pf_step, so the results are bitwise
 * those of separate pf_run calls.  Contexts of other patch sizes, and
 * contexts of 512 or more PEs per filter (whose iterations end with a
 * once-per-filter master step launch, which a group does not have) are
 * stepped one by one inside the same run.  The contexts must use one stream and stay
 * alive until pf_batch_destroy; the batch owns only its launch tables. */
typedef struct pf_batch pf_batch;
int pf_batch_create(pf_ctx *const *ctxs, uint32_t n, pf_batch **out);

/* n_steps iterations of every context: context i takes its frames from
 * d_frames[i] + s * frame_stride[i] (host arrays of n device pointers and
 * strides in floats).  use_graph != 0 runs the batched contexts as HIP
 * graphs, in runs of at most 64 iterations: the launches of a run of a given
 * length are captured once per batch and replayed (their arguments are read
 * from the batch's device table, which each run rewrites); the ring tables
 * are rebuilt ahead of a run when needed, and the contexts without a batched
 * variant run beside the graph.  Either way the launches are only enqueued
 * (the call synchronizes the stream before it rewrites the argument table).
 * PF_ESTATE if a context is recording a gradient. */
int pf_batch_run(pf_batch *b, const float *const *d_frames, const uint64_t *frame_stride,
                 uint32_t n_steps, int use_graph);

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): pf_batch_run without a graph, its
 * argument table staged in a fixed device array of PF_BATCH_NOALLOC_MAX_ARGS
 * entries (one per batched context and iteration, about 1 MiB) that the
 * library holds on each GPU until the process ends, instead of a buffer the
 * batch grows with hipMalloc.  The call allocates no device memory.
 * n_steps x (contexts launched in groups) above PF_BATCH_NOALLOC_MAX_ARGS
 * gives PF_EUNSUPPORTED before anything is enqueued.  The array is shared by
 * every call on that GPU and keeps the last call's table: a call waits for
 * the batch's stream before it overwrites the table, so calls on one stream
 * are ordered, but calls that overlap on one GPU from different streams or
 * threads race.  PF_EHIP if the array's address could not be taken when
 * the contexts were created. */
#define PF_BATCH_NOALLOC_MAX_ARGS 4096
int pf_batch_run_noalloc(pf_batch *b, const float *const *d_frames, const uint64_t *frame_stride,
                         uint32_t n_steps);
void pf_batch_destroy(pf_batch *b);

/* ------------------------------------------------------------- gradient */
/* The filter's estimate of the log marginal likelihood of a run of K
 * iterations is, per filter, J = sum_k (log W_k - log N_p), with W_k the sum
 * of the PE masses of Alg. 3 step 9 (the carried weights are renormalized by
 * W_{k-1} in step 4, so the increments chain).  With every discrete choice of
 * the run held fixed -- ring, N_ex, exchanged slots, the ancestors of step 7
 * and the patch positions of the likelihood -- and the normals fixed by their
 * counters, J is a smooth function of theta = (psf_sigma, I0, q); I0 shifts
 * the intensity of every particle of the state the recording starts from
 * (for a recording that starts at pf_init with the tracking start, that is
 * the true initial intensity).
 *
 * pf_grad_begin starts recording: the next max_steps iterations (pf_step /
 * pf_run) keep their propagated particles, ancestors and PE records on the
 * device ((max_steps + 1) x (22 N + 56 F M) bytes, kept for reuse until
 * pf_destroy).  Patch likelihood and N_p <= PF_MAX_PER_PE_LDS only
 * (PF_EUNSUPPORTED otherwise); q must be
 * positive (PF_EINVAL).  PF_ESTATE while recording or after pf_exchange.
 * An iteration beyond max_steps returns PF_ESTATE and does nothing. */
int pf_grad_begin(pf_ctx *c, uint32_t max_steps);

/* While recording: host_J (host double [F]) receives J over the iterations
 * recorded so far.  Synchronizes the stream.  PF_ESTATE if not recording. */
int pf_grad_value(pf_ctx *c, double *host_J);

/* Run the reverse sweep over the recorded iterations and stop recording.
 * d_frames: the recorded iterations' frames again, d_frames + i * frame_stride
 * for the i-th recorded iteration (device float32, caller-owned).
 * host_out (host double [F][4]) receives per filter (J, dJ/dpsf_sigma,
 * dJ/dI0, dJ/dq).  Synchronizes the stream; the context then continues from
 * the last recorded iteration.  PF_ESTATE if not recording. */
int pf_grad_end(pf_ctx *c, const float *d_frames, uint64_t frame_stride, double *host_out);

/* Free everything the context owns (synchronizes its stream first). */
void pf_destroy(pf_ctx *c);

/* Static text for a PF_* code. */
const char *pf_strerror(int code);

/* ------------------------------------------------------------------ debug */
/* Buffers readable with pf_debug_get (host_dst must hold `bytes` bytes; the
 * required size is returned through pf_debug_size).  TRACE buffers describe
 * the last completed iteration and need PF_DEBUG_TRACE. */
enum {
    PF_DBG_STATE = 0,      /* float  [5][N] resampled particles */
    PF_DBG_LOGMASS = 1,    /* double [F][M] log W^(m)_k */
    PF_DBG_PE_RECORDS = 2, /* pf_pe_record [F][M] */
    PF_DBG_RING = 3,       /* uint32 [F][M] pred(m) of the last iteration      (TRACE) */
    PF_DBG_NEX = 4,        /* uint32 [F] N_ex of the last iteration */
    PF_DBG_SRC = 5,        /* int64  [N] exchange source map                   (TRACE) */
    PF_DBG_PROP = 6,       /* float  [5][N] propagated particles               (TRACE) */
    PF_DBG_ELL = 7,        /* float  [N] log-likelihood of each slot           (TRACE) */
    PF_DBG_Q = 8,          /* uint32 [N] fixed-point weights                   (TRACE) */
    PF_DBG_ANCESTORS = 9,  /* uint32 [N] ancestor slot within the PE           (TRACE) */
    PF_DBG_V = 10,         /* uint32 [F][M] systematic offsets                 (TRACE) */
    PF_DBG_LAMBDA = 11,    /* float  [N] carried log-weight of each slot       (TRACE) */
    PF_DBG_LINEAGE = 12    /* int32  [N] lineage tags                          (LINEAGE) */
};
size_t pf_debug_size(const pf_ctx *c, int which);
int pf_debug_get(pf_ctx *c, int which, void *host_dst, size_t bytes);

/* Overwrite the particles (host float [5][N]) and the PE log-weights (host
 * double [F][M], NULL = all zero), and declare `step` iterations completed.
 * Restores a checkpoint taken with pf_debug_get(STATE / LOGMASS). */
int pf_debug_set_state(pf_ctx *c, const float *host_state, const double *host_log_mass,
                       uint64_t step);
/* Set the lineage tags (host int32 [N]); needs PF_DEBUG_LINEAGE. */
int pf_debug_set_lineage(pf_ctx *c, const int32_t *host_tags);

/* Replay of another run's discrete choices (test support): the next iteration
 * takes its ancestors from d_anc (device uint32 [N], ancestor slot within the
 * PE, non-decreasing within each PE) instead of step 7, and N_ex from d_nex
 * (device uint32 [F]) instead of step 2; either may be NULL.  The pointers are
 * read by that iteration only (they must stay valid until the stream has
 * passed it) and are then forgotten. */
int pf_debug_force_next(pf_ctx *c, const uint32_t *d_anc, const uint32_t *d_nex);

/* The device integer stages on host arrays, run synchronously on the current
 * device with the same device code as pf_step. */
/* Systematic resampling (Alg. 3, step 7) of n_blocks independent PEs of
 * n_p <= PF_MAX_PER_PE_LDS particles (the LDS kernel's stage):
 * q [n_blocks][n_p] fixed-point weights, v [n_blocks] offsets (v < sum q),
 * anc_out [n_blocks][n_p] ancestors a_j = min{i : n_p C_i > j T + v}. */
int pf_debug_resample_q(const uint32_t *q, uint32_t n_blocks, uint32_t n_p, const uint32_t *v,
                        uint32_t *anc_out);
/* Exchange count (Alg. 3, step 2; Eq. 3 and 4) from integer PE masses p[M]. */
int pf_debug_nex(const uint32_t *p, uint32_t M, uint32_t n_p, uint32_t mode, float fixed_ratio,
                 float initial_ratio, float eff_cutoff, int first_iteration, uint32_t *nex_out);
/* Ring of iteration k of filter f (Alg. 3, step 1): pred_out[M]. */
int pf_debug_ring(uint64_t seed, uint32_t f, uint32_t k, uint32_t M, uint32_t mode,
                  uint32_t groups, uint32_t *host_pred_out);
/* Philox4x32-10 of n counters: ctr [n][4], key [2], out [n][4]. */
int pf_debug_philox(const uint32_t *ctr, const uint32_t *key, uint32_t n, uint32_t *out);

#ifdef __cplusplus
}
#endif

#endif /* ARNA_H */
