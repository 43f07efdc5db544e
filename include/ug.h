/*
 * ug.h -- C-ABI of libug: an urgency-gated launcher for deadline-bound task
 * chains of GPU kernels on one MI355X (gfx950), after UrgenGo
 * (arXiv 2509.12207).
 *
 * Problem statement (Sec. 1, Sec. 2 "Urgency Level", Sec. 4.2): a set of
 * periodic task chains shares one GPU.  Each chain has an end-to-end deadline
 * D and an ordered list of tasks; each task is a CPU segment followed by a
 * sequence of GPU kernels that run on one stream.  Every arriving data frame
 * starts an instance of its chain.  The library launches the kernels of all
 * instances itself, ordered by the urgency of Eq. (2), with task-level stream
 * binding (Sec. 4.4.3), delayed launching (Sec. 4.4.4) and batched launch
 * synchronisation with batch overlap (Sec. 4.4.5), and reports each frame's
 * latency and deadline miss (Sec. 6.2).
 *
 * Conventions
 *   - Every function is extern "C" and never throws.  Functions returning
 *     ug_status return UG_OK (0) or a negative UG_E* code; the message of the
 *     last failure on a context is available from ug_last_error().
 *   - Times are int64 nanoseconds on CLOCK_MONOTONIC (ug_now_ns()).
 *   - Buffers are device pointers (hipMalloc or torch allocations on the
 *     context's device).  The library never allocates or frees them.
 *   - A device error (a failed HIP call) is sticky: once reported, every later
 *     call on the context returns UG_EDEVICE.
 *
 * Threading: one caller thread may call ug_frame_submit / ug_poll_complete /
 * ug_drain while the context's internal gate thread runs.  Other calls must
 * not overlap with them.
 */
#ifndef UG_H
#define UG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define UG_ABI_VERSION 7u

typedef int32_t ug_status;
enum {
  UG_OK = 0,
  UG_EINVAL = -1,    /* invalid argument (shape, slot, id, size, null)       */
  UG_ENOMEM = -2,    /* host or device allocation failed                     */
  UG_EDEVICE = -3,   /* a HIP call failed; sticky for the context            */
  UG_EAGAIN = -4,    /* submission queue full; retry after polling           */
  UG_ETIMEDOUT = -5, /* ug_drain timed out                                   */
  UG_ESTATE = -6,    /* call not allowed in the context's current state      */
  UG_ENODEV = -7     /* the context has no device (created with device < 0) */
};

/* Launch policy. */
enum {
  UG_POLICY_FIFO = 0,    /* plain launch: every kernel of a ready task at once,
                            on that task's own stream, one end event per task
                            (the "vanilla" baseline of Sec. 6.3)             */
  UG_POLICY_URGENCY = 1  /* urgency-ordered gate of Sec. 4.4                  */
};

/* Switches of the urgency policy (ug_config.flags). */
enum {
  UG_F_BIND = 1u,      /* task-level stream binding with reservation (4.4.3) */
  UG_F_DELAY = 2u,     /* delayed launching (4.4.4)                          */
  UG_F_BATCH = 4u,     /* batched launching with batch overlap (4.4.5)       */
  UG_F_CALIBRATE = 8u, /* record highest-urgency samples for TH_urgent (4.4.3) */
  UG_F_ADMIT = 16u,    /* urgency-ordered admission: a task that is not truly
                          urgent starts only while fewer than admit_tasks
                          instances have kernels in flight (stands in for
                          stream priorities, see ug_config)               */
  UG_F_EXIT = 32u,     /* early chain exit (Sec. 4.3): a frame whose urgency
                          is negative when a task would start leaves the
                          chain; it completes as missed and exited        */
  UG_F_NO_OVERLAP = 64u, /* launch-synchronisation variants (Sec. 6.4): a
                          closed batch is waited for until it has finished
                          (not until it has started) before the task's next
                          batch is launched.  With UG_F_BATCH: synchronous
                          batched launching; with delta_eval_ns = 0 as well:
                          synchronous launching (one kernel per batch).
                          UG_F_BATCH alone off: asynchronous launching     */
  UG_F_GRAPH = 128u,    /* task graphs (configuration 2): every task of a frame
                          is captured once (per buffer set and per-frame
                          sizes) into a HIP graph and launched as one graph
                          on its bound stream; the gate decides per task
                          (delayed launching at the task's first kernel,
                          with the task's largest utilisation; no batches
                          inside a task).  Applies to both policies.      */
  UG_F_CPU_PRIO = 512u, /* urgency-centric CPU scheduling (Sec. 4.3), with
                          ug_config.cpu_cores > 0: whenever a chain starts a
                          CPU segment, every active instance is ranked by
                          urgency, and the cores run the segments of the
                          best ranks, preempting worse ones (fixed
                          priorities, as SCHED_FIFO); without it the cores
                          serve segments first come, first served      */
  UG_F_FUSE = 1024u,    /* fused tails (configuration 2): the bias+ReLU
                          after a contraction, with the row softmax and row
                          sum of its output, runs as one work item of the
                          tail executor (ug_tails_*) instead of as launches:
                          the contraction counts its finished wavefronts on
                          the device, the item is served from a device-side
                          queue ordered by the gate's current urgency rank
                          of its instance (Sec. 4.2), and the task's events
                          count as observed only once the items published
                          before them have finished.  A tail qualifies by
                          the rule of ug_chain_tails; others launch as
                          usual.  Applies to both policies (FIFO: items in
                          publication order).  Decided at attach (the pool
                          needs extra streams, see ug_streams_needed).    */
  UG_F_PLACE = 256u     /* queue placement of the stream pool: when streams
                          are attached (or created), the library measures
                          which hardware queue each one uses and assigns
                          lanes (FIFO: task streams) round-robin over the
                          queues, so that the first lanes of every level
                          never share a queue while another is free.
                          Applies to both policies; decided at attach.    */
};

/* Orders that rank the instances (ug_config.order_key).  The paper's
 * urgency (Eq. 2) is the default; the others are the alternatives of its
 * policy comparison (Sec. 6.4), each with ties broken by (chain, frame):
 *   EDF   earliest absolute deadline t_arr + D first;
 *   SJF   least remaining estimated work (GPU and CPU, as in Eq. 2) first;
 *   HRRN  highest response ratio (t - t_arr + R) / R first, R = remaining
 *         work (R = 0 ranks first);
 *   LCUF  lowest chain utilisation (a frame's estimated work / period)
 *         first (period 0 ranks last);
 *   SAEDF, EQDF  earliest deadline of the instance's current task, where
 *         the chain's remaining slack S = t_arr + D - t_ref - W (t_ref: the
 *         task's start, W: the estimated work of it and every later task)
 *         is split over the remaining m tasks equally (SAEDF: S / m) or in
 *         proportion to each task's estimated work w (EQDF: S w / W); the
 *         task's deadline is t_ref + w + its share.  The paper names these
 *         two by citation only; this is the reading built.
 * The key replaces urgency in the service order, the binding rank and the
 * "more urgent than" of delayed launching; truly urgent (TH_urgent), the
 * reserved level and calibration stay defined by urgency.  Best-effort
 * instances rank last under every key. */
enum {
  UG_KEY_URGENCY = 0,
  UG_KEY_EDF = 1,
  UG_KEY_SJF = 2,
  UG_KEY_HRRN = 3,
  UG_KEY_LCUF = 4,
  UG_KEY_SAEDF = 5,
  UG_KEY_EQDF = 6
};

/* Operations.  Shapes and slot meaning per op; all float buffers are fp32,
 * row-major / NCHW, densely packed.  "in"/"out" hold buffer-slot indices
 * into the pointer array passed with each frame (-1 = unused).
 *
 *  UG_OP_GEMM_F32       C = A B.  shape {M, N, K}; in {A[M,K], B[K,N]};
 *                       out {C[M,N]}.  FP32 MFMA, FP32 accumulation.
 *  UG_OP_BIAS_RELU_F32  y = max(x + b, +0).  shape {R, C, axis}; in {X[R,C],
 *                       b}; out {Y[R,C]} (Y may alias X).  axis 0: b[C] per
 *                       column; axis 1: b[R] per row (NCHW channel bias).
 *  UG_OP_CONV3X3_F32    3x3 cross-correlation, stride 1, zero pad 1, as many
 *                       output as input channels.  shape {N, C, H, W},
 *                       H * W < 2^26, 9 C^2 < 2^33; in {X[N,C,H,W],
 *                       W[C,C,3,3]}; out {Y[N,C,H,W]}.
 *  UG_OP_ROWSUM_F32     r_i = sum_j Z_ij.  shape {R, C}; in {Z[R,C]}; out {r[R]}.
 *  UG_OP_SOFTMAX_F32    row softmax.  shape {R, L}; in {X[R,L]}; out {Y[R,L]}
 *                       (Y may alias X).
 *  UG_OP_VOXEL_F32      bird's-eye-view pillar binning.  shape {N, nx, ny};
 *                       fparam {xmin, ymin, scale}; in {pts[N,4] (x,y,z,i)};
 *                       out {vidx[N] int32, count[nx*ny] int32,
 *                       zmax[nx*ny] fp32, first[nx*ny] int32}.  Cell of a
 *                       point: ix = floor(fl32(fl32(x - xmin) * scale)), iy
 *                       likewise, inside iff 0 <= ix < nx and 0 <= iy < ny;
 *                       vidx = iy*nx + ix or -1.  Empty cells: count 0,
 *                       zmax -inf, first -1.  z must not be NaN.
 *  UG_OP_GEMM_FP8       C = A B with A, B in OCP FP8 E4M3 (one byte per
 *                       value) and an FP32 result, FP32 accumulation on the
 *                       FP8 matrix cores.  shape {M, N, K, m0}, K a multiple
 *                       of 16; in {A[m0+M,K] row-major, Bt[N,K] = B
 *                       transposed (K contiguous)}; out {C[m0+M,N] fp32}:
 *                       rows m0 .. m0+M-1 of C from the same rows of A
 *                       (m0 = 0: the whole product; m0 > 0: one row band of
 *                       a product split into sub-kernels, the kernel
 *                       splitting of the cCUDA baseline, Sec. 6.3); A and
 *                       Bt 16-byte aligned.  The best-effort load of an
 *                       overloaded GPU.
 *  UG_OP_GEMM_BF16      C = A B with A, B in bfloat16 (two bytes per value,
 *                       the upper half of an IEEE binary32) and an FP32
 *                       result, FP32 accumulation on the BF16 matrix cores.
 *                       shape {M, N, K}, K a multiple of 32 below 2^30;
 *                       in {A[M,K] row-major, Bt[N,K] = B transposed};
 *                       out {C[M,N] fp32}; A and Bt 16-byte aligned.  The
 *                       reduced-precision form of the GEMM (configuration
 *                       with BF16 contractions).
 *  UG_OP_CONV3X3_BF16   the 3x3 convolution of UG_OP_CONV3X3_F32 on bfloat16
 *                       operands, FP32 result, FP32 accumulation on the
 *                       BF16 matrix cores.  shape {1, C, H, W}, C a multiple
 *                       of 32 (<= 8192); in {X[H,W,C] (NHWC, channels
 *                       innermost), W[C,3,3,C] (OHWI)}; out {Y[C,H,W] fp32
 *                       NCHW}; X and W 16-byte aligned.
 *  UG_OP_VECADD_F32     c = a + b (one float32 addition each).  shape {N, W,
 *                       R}; in {A[N], B[N]}; out {C[N]}; run by exactly W
 *                       workgroups of 256 lanes (1 <= W <= 65536), the pass
 *                       repeated R times (0 or 1: once; <= 65536), so its
 *                       utilisation is min(1, W / CUs) and its duration
 *                       follows from N R / W: the custom kernel of the
 *                       utilisation and kernel-time experiments (Sec. 6.6).
 */
enum {
  UG_OP_GEMM_F32 = 1,
  UG_OP_BIAS_RELU_F32 = 2,
  UG_OP_CONV3X3_F32 = 3,
  UG_OP_ROWSUM_F32 = 4,
  UG_OP_SOFTMAX_F32 = 5,
  UG_OP_VOXEL_F32 = 6,
  UG_OP_GEMM_FP8 = 7,
  UG_OP_GEMM_BF16 = 8,
  UG_OP_VECADD_F32 = 9,
  UG_OP_CONV3X3_BF16 = 10,
  UG_OP_UPLOAD_H2D = 11,
  UG_OP_ACCUM_I32 = 12
};

/* One kernel of a task (a row of the paper's lookup table, Tab. "Example
 * lookup table", plus its buffer bindings).  UPLOAD_H2D is a host-to-device
 * copy (the cuMemCpy row of Tab. "Intercepted function calls": delayed like
 * a launch, bound to the task's stream; its utilisation is taken as 1 unless
 * given).  shape {N, unit bytes}; in {source: host memory the caller pinned
 * (hipHostMalloc, torch pin_memory)}; out {device destination}; copies
 * N * unit bytes.  ACCUM_I32 updates device-resident chain state: state_i +=
 * x_i in int32 (wrapping); shape {N}; in {x[N]}; out {state[N]}, a buffer
 * every frame of the chain shares, updated in frame order. */
typedef struct {
  int32_t op;          /* UG_OP_*                                             */
  int32_t in[3];       /* input buffer slots, -1 = unused                     */
  int32_t out[4];      /* output buffer slots, -1 = unused                    */
  int64_t shape[4];    /* op-specific, see above                              */
  float fparam[4];     /* op-specific float parameters                        */
  int64_t est_ns;      /* estimated execution time E_k; 0 = not yet profiled  */
  float util;          /* utilisation U_k in [0,1]; < 0 = derive from launch  */
  int32_t frame_dim;   /* 0: fixed shape.  d in 1..4: a per-frame size: each
                          frame gives a value v as dims[d-1] in
                          ug_frame_submit_dims, and s = v >> frame_shift
                          sets the op's frame dimension (below); the
                          registered shape is the largest (the size its
                          buffers and workspace are made for)            */
  int32_t frame_shift; /* 0..30 (see frame_dim)                             */
  int32_t pad0;
} ug_kernel;

/* The frame dimension each op takes from s = v >> frame_shift (other ops
 * take no per-frame size: registration fails with UG_EINVAL):
 *   VOXEL_F32     N = s points (s may be 0)
 *   UPLOAD_H2D    N = s units (s may be 0)
 *   GEMM_F32      M = s rows          SOFTMAX_F32   R = s rows
 *   CONV3X3_*     H = W = s (registered square)
 *   BIAS_RELU_F32 axis 1: C = s * s (the image plane of a channel);
 *                 axis 0: R = s rows
 *   ROWSUM_F32    C = s * s (each row is an image plane)
 * The estimate E_k of such a kernel follows the frame's size through its
 * profile points (ug_kernel_set_profile). */

/* One task: a CPU segment (host-side time before the kernels may launch,
 * Sec. 4.2) followed by kernels that run in order on one stream. */
typedef struct {
  const ug_kernel* kernels;
  uint32_t n_kernels;
  uint32_t pad0;
  int64_t cpu_ns;      /* CPU-segment time; also its estimate in Eq. (2)     */
} ug_task;

typedef struct {
  uint32_t abi_version;    /* must be UG_ABI_VERSION                         */
  int32_t policy;          /* UG_POLICY_*                                    */
  uint32_t flags;          /* UG_F_* (urgency policy only)                   */
  int32_t device;          /* HIP device ordinal; < 0 = no device: the
                              context only registers chains and replays
                              decision instants (ug_replay_instant)          */
  int64_t delta_eval_ns;   /* Delta_eval of batched launching (0.5 ms)       */
  int64_t delay_poll_ns;   /* sleep step of delayed launching (1 ms);
                              0 = re-check a held launch at every instant    */
  float util_exempt;       /* kernels with U below this are never held (0.1) */
  int32_t n_levels;        /* stream levels, 1..8; level 0 is reserved for
                              truly urgent tasks when n_levels > 1          */
  int32_t lanes[8];        /* streams per level                             */
  int64_t th_slack_ns;     /* TH_urgent carried as a slack: truly urgent iff
                              0 <= slack < th_slack_ns; <= 0 = nobody        */
  int64_t idle_sleep_ns;   /* gate thread sleep when idle; 0 = spin         */
  uint32_t queue_capacity; /* max frames submitted and not yet completed    */
  uint32_t trace_capacity; /* decision-log records kept; 0 = no log         */
  int64_t calib_period_ns; /* with UG_F_CALIBRATE: the highest urgency among
                              active kernels is recorded at the first instant
                              at or after each sampling time, one period
                              apart (Sec. 4.4.3, 1 ms); 0 = every instant    */
  int64_t admit_tasks;     /* with UG_F_ADMIT: instances with kernels in
                              flight before new tasks wait (4)              */
  uint64_t hbm_budget_bytes; /* serving admission: the device memory the
                              frames in flight may hold, by the footprints
                              set with ug_chain_set_footprint; a submission
                              that would exceed it returns UG_EAGAIN.
                              0 = no budget                                  */
  int32_t order_key;       /* UG_KEY_* (urgency policy only; default URGENCY) */
  int32_t est_noise_permille; /* estimate-noise experiment (Sec. 6.6): n in
                              0..1000; the estimates of task j of frame f of
                              chain c enter the urgency (and SJF / HRRN) as
                              E * (1000 + k) / 1000, k uniform in [-n, n]
                              drawn by SplitMix64 from (noise_seed, c, f, j);
                              batching keeps the profiled E.  0 = none      */
  uint64_t noise_seed;
  int64_t max_hold_ns;     /* hold-age bound (urgency policy): once a task
                              has waited this long since its first hold
                              (delayed launching or admission), it is not
                              held again; a timer re-decides it when the
                              bound is reached.  Best-effort tasks
                              (deadline 0) are not bounded.  0 = no bound
                              (the paper)                                   */
  int32_t own_streams;     /* 0: the caller provides the stream pool with
                              ug_attach_streams before ug_start (streams made
                              by torch); 1: the library creates its own
                              default-priority streams at ug_start          */
  int32_t cpu_cores;       /* CPU cores the tasks' CPU segments share (Sec.
                              4.1: a segment runs on a core for its CPU time,
                              one segment per core); 0 = every segment runs
                              at once (no CPU contention).  0..1024 */
  uint32_t fuse_workers;   /* with UG_F_FUSE: worker workgroups of the tail
                              executor (1..1024, 64)                        */
  int32_t pad1;
  int64_t fuse_idle_ns;    /* with UG_F_FUSE: the executor leaves after this
                              long without progress, and is launched again
                              when items are pending (500 us)               */
  const char* tile_table;  /* a tile-variant table file (ug_tile_load) read
                              by ug_create into the process-wide table, or
                              NULL                                           */
} ug_config;

/* Completion of one frame (Sec. 6.2: latency, miss). */
typedef struct {
  uint32_t chain;
  uint32_t pad0;
  uint64_t frame;          /* frame index within its chain (0, 1, ...)      */
  int64_t t_arr_ns;
  int64_t t_done_ns;       /* when the gate observed the last kernel done   */
  int64_t latency_ns;      /* t_done - t_arr                                */
  int32_t missed;          /* latency > deadline, or exited                 */
  int32_t n_holds;         /* launches of this frame that were held         */
  int32_t n_batches;       /* launch batches of this frame                  */
  int32_t exited;          /* left the chain early (UG_F_EXIT); t_done is
                              the time it left, its later tasks never ran    */
} ug_completion;

/* Decision-log record.  The log is a sequence of instants; each INSTANT
 * record is followed by its inputs (ARRIVE with its DIMS, EVDONE) and then
 * the decisions taken at that instant (COMPLETE, TSTART, BIND, HOLD, EVREC,
 * LAUNCH).
 *   INSTANT  t = instant time, a = #arrivals, b = #observed events
 *   ARRIVE   chain, frame, t = t_arr
 *   DIMS     chain, frame, a = index d, t = the frame's dims[d] (after the
 *            frame's ARRIVE; frames submitted with per-frame sizes)
 *   EVDONE   chain, frame, task, a = kind (0 batch start, 1 task end), b = seq
 *   COMPLETE chain, frame, t = t_done
 *   EXIT     chain, frame, task, t: the frame leaves its chain instead of
 *            starting task (early chain exit)
 *   TSTART   chain, frame, task
 *   BIND     chain, frame, task, a = level, b = lane
 *   HOLD     chain, frame, kernel
 *   EVREC    chain, frame, task, a = kind, b = seq (batch index, or the
 *            number of batches for the end event)
 *   LAUNCH   chain, frame, kernel, a = level, b = lane
 *   CPU      chain, frame, task, a = 1: the task's CPU segment takes a core,
 *            0: it loses its core to a better-ranked one (cpu_cores > 0)
 * kernel = index within the chain (all tasks' kernels numbered in order). */
enum {
  UG_REC_INSTANT = 1, UG_REC_ARRIVE = 2, UG_REC_EVDONE = 3, UG_REC_COMPLETE = 4,
  UG_REC_TSTART = 5, UG_REC_BIND = 6, UG_REC_HOLD = 7, UG_REC_EVREC = 8,
  UG_REC_LAUNCH = 9, UG_REC_EXIT = 10, UG_REC_DIMS = 11, UG_REC_CPU = 12
};
typedef struct {
  int32_t type;
  int32_t chain;
  int64_t frame;
  int32_t task;
  int32_t kernel;
  int32_t a;
  int32_t b;
  int64_t t;
} ug_record;

typedef struct {
  uint64_t frames_submitted;
  uint64_t frames_completed;
  uint64_t frames_missed;
  uint64_t launches;
  uint64_t holds;
  uint64_t batches;
  uint64_t instants;
  uint64_t collisions;     /* truly urgent launches made while another
                              chain's kernels were active (Sec. 6.4)        */
  int64_t decide_ns;       /* time spent deciding (policy only)             */
  int64_t launch_ns;       /* time spent in HIP launch/record calls         */
  uint64_t trace_records;  /* records currently in the log                  */
  uint64_t trace_dropped;  /* records lost because the log was full         */
  uint64_t frames_deferred; /* submissions refused by the HBM budget        */
  uint64_t hbm_peak_bytes; /* largest footprint of the frames in flight     */
  uint64_t tails_fused;    /* tails published to the tail executor (FUSE)   */
  uint64_t tails_unfused;  /* qualifying tails launched as kernels (no free
                              slot, or buffers not 16-byte aligned)          */
  uint64_t executor_launches; /* launches of the tail executor              */
  uint64_t collision_hist[8]; /* collisions by the number of other chains'
                              instances with kernels in flight: 1, 2, ...,
                              7, and 8 or more (Sec. 6.4)                  */
} ug_stats;

/* ------------------------------------------------------------------------ */

/* Fills *cfg with the defaults: URGENCY with BIND|DELAY|BATCH (Sec. 4.4.3-
 * 4.4.5) plus ADMIT and PLACE, Delta_eval 0.5 ms (Sec. 4.4.5), 1 ms sleep
 * step (Sec. 4.4.4), U exemption 0.1 (the paper's values), device 0,
 * 2 levels with lanes {2, 6} (the reserved level and one shared level: all
 * streams have the same hardware priority, so further levels only split
 * lanes), no truly-urgent threshold, spinning gate thread. */
void ug_config_default(ug_config* cfg);

/* CLOCK_MONOTONIC in ns: the clock of every time argument (arrival times
 * and the elapsed time of Eq. 2). */
int64_t ug_now_ns(void);

/* Static text of a status code (never NULL). */
const char* ug_status_str(ug_status s);

/* Creates a context: one gate (its policy, Active Kernel Buffer and event
 * pool) for the chains that will share one GPU (the system of Sec. 3 and
 * Sec. 4.4).  cfg is copied.  With cfg->device >= 0 it creates a pool of
 * events on that device; the streams come from ug_attach_streams (or, with
 * own_streams, are created at ug_start).  *out is owned by the caller and
 * released with ug_destroy.  Errors: UG_EINVAL (a field out of range, wrong
 * abi_version), UG_ENOMEM, UG_EDEVICE (no such device, event creation). */
ug_status ug_create(const ug_config* cfg, void** out);

/* Stops the gate thread (without waiting for in-flight frames), waits for
 * every stream of the pool to drain, then releases events, task graphs,
 * kernel workspaces and the streams the library created itself (attached
 * streams stay the caller's).  Buffers of unfinished frames are left
 * untouched. */
void ug_destroy(void* ctx);

/* Message of the last error on ctx; with ctx NULL, the message of the last
 * failed ug_create in the process.  The text is a copy owned by the calling
 * thread, valid until that thread's next ug_last_error call; any thread may
 * call it while others fail calls on the same context. */
const char* ug_last_error(void* ctx);

/* Registers a chain: a period (informational), an end-to-end deadline and
 * an ordered task list (Sec. 4.1).  deadline_ns = 0 registers a best-effort
 * chain (background load with no deadline): it has no urgency (ranked below
 * every deadline instance), is never truly urgent, all its kernels are
 * subject to delayed launching whatever their utilisation, it is not sampled
 * for TH_urgent, and its frames complete with missed = 0 and stay out of
 * ug_get_metrics.  n_buffers is the number of buffer slots
 * each frame supplies.  Descriptors are deep-copied; the device workspace a
 * kernel needs (ug_kernel_workspace) is allocated here, never on the launch
 * path, and released by ug_destroy.  Only before ug_start.  Errors:
 * UG_EINVAL (bad op/shape/slot, deadline < 0), UG_ESTATE (already started),
 * UG_ENOMEM. */
ug_status ug_chain_register(void* ctx, int64_t period_ns, int64_t deadline_ns,
                            const ug_task* tasks, uint32_t n_tasks,
                            uint32_t n_buffers, uint32_t* chain_id);

/* Sets / reads the estimate E_k and utilisation U_k of kernel `kernel` of a
 * chain (offline profile, Sec. 4.1 and Tab. "Example lookup table").  Set
 * only before ug_start.  util < 0 keeps the current value. */
ug_status ug_kernel_set_estimate(void* ctx, uint32_t chain, uint32_t kernel,
                                 int64_t est_ns, float util);
ug_status ug_kernel_get_estimate(void* ctx, uint32_t chain, uint32_t kernel,
                                 int64_t* est_ns, float* util);

/* Profile points of a kernel with a per-frame size (frame_dim > 0): its
 * estimate at n frame values v[i] (strictly increasing) is e[i] ns.  A frame
 * of value v then enters Eq. 2 and the batch sums with the estimate at v:
 * linear between neighbouring points (rounded down), the end point's
 * estimate beyond either end -- the lookup of Sec. 4.1 / Tab. "Example
 * lookup table" keyed by launch size.  n = 0 removes the points (the fixed
 * E_k applies).  ug_profile sets them.  Only before ug_start.  Errors:
 * UG_EINVAL (no such kernel, no frame_dim, n > 16, v not increasing, e < 0),
 * UG_ESTATE.  get: copies up to cap points and sets *n to their number. */
ug_status ug_kernel_set_profile(void* ctx, uint32_t chain, uint32_t kernel,
                                const int64_t* v, const int64_t* e, uint32_t n);
ug_status ug_kernel_get_profile(void* ctx, uint32_t chain, uint32_t kernel,
                                int64_t* v, int64_t* e, uint32_t cap, uint32_t* n);

/* Offline profiling stage (Sec. 4.1): runs every kernel of the chain in
 * isolation on the given frame buffers (warmup, then reps timed with HIP
 * events; the median is E_k) and stores the estimates.  A kernel with a
 * per-frame size is measured at the largest frame value and at 1/2, 1/4 and
 * 1/8 of it (its profile points; E_k is the largest).  Kernels with the
 * same (op, shape) share one measurement.  Overwrites the buffers' contents.
 * Only before ug_start.  Errors: UG_ENODEV, UG_EINVAL, UG_EDEVICE. */
ug_status ug_profile(void* ctx, uint32_t chain, void* const* buffers,
                     uint32_t n_buffers, uint32_t warmup, uint32_t reps);

/* Changes TH_urgent (as a slack; Sec. 4.4.3) or the policy's switches (the
 * mechanisms of Sec. 4.4.3-4.4.5 and calibration sampling).  Only while not
 * started; the policy itself is fixed at creation.  Errors: UG_EINVAL,
 * UG_ESTATE. */
ug_status ug_set_threshold(void* ctx, int64_t th_slack_ns);
ug_status ug_set_flags(void* ctx, int32_t policy, uint32_t flags);

/* Starts the gate thread, which runs the decision instants of Sec. 4.4
 * (urgency evaluation, binding, delayed and batched launching) until
 * ug_stop.  Registration is closed from here on.  Errors: UG_ENODEV,
 * UG_ESTATE (already started; no streams attached and own_streams 0),
 * UG_EDEVICE. */
ug_status ug_start(void* ctx);

/* Submits one frame of `chain` arriving at t_arr_ns (< 0: now; a future time
 * is honoured: the frame arrives when the clock reaches it): a data frame
 * that starts an instance of the chain (Sec. 4.2, the arrival that sets
 * t_arr in Eq. 2).  Non-blocking.  buffers[i] is
 * the device pointer of slot i; the caller keeps them alive and unmodified
 * until the frame is returned by ug_poll_complete (borrowed).  *frame gets
 * the frame index within the chain.  Errors: UG_EINVAL (also: the chain has
 * per-frame sizes, see ug_frame_submit_dims), UG_ESTATE (not started),
 * UG_EAGAIN (queue_capacity frames outstanding, or the HBM budget would be
 * exceeded), UG_EDEVICE. */
ug_status ug_frame_submit(void* ctx, uint32_t chain, int64_t t_arr_ns,
                          void* const* buffers, uint32_t n_buffers,
                          uint64_t* frame);

/* ug_frame_submit for chains whose kernels have per-frame sizes
 * (ug_kernel.frame_dim): dims[d] is this frame's value of every shape[0]
 * registered with frame_dim = d + 1 (n_dims covers the chain's largest
 * frame_dim; each value at least 1, or 0 for the voxel scatter, and at most
 * the registered shape[0]).  Serving form (configuration with per-frame
 * point counts).  Errors: those of ug_frame_submit; UG_EINVAL also for
 * dims out of range. */
ug_status ug_frame_submit_dims(void* ctx, uint32_t chain, int64_t t_arr_ns,
                               void* const* buffers, uint32_t n_buffers,
                               const int64_t* dims, uint32_t n_dims,
                               uint64_t* frame);

/* Device memory (bytes) one frame of `chain` holds from submission until
 * its completion is delivered, for admission against
 * ug_config.hbm_budget_bytes (serving form, device-resident frames).
 * Default 0 (not counted).  A frame whose footprint would take the frames
 * in flight past the budget is refused with UG_EAGAIN (nothing is queued:
 * the caller retries after completions).  Only before ug_start.  Errors:
 * UG_EINVAL, UG_ESTATE. */
ug_status ug_chain_set_footprint(void* ctx, uint32_t chain, uint64_t bytes);

/* Number of streams ug_attach_streams expects: the sum of ug_config.lanes
 * (urgency policy: the stream pool of Sec. 4.4.3, level by level), or one
 * per task of every registered chain (FIFO launch: each task on its own
 * stream, the baseline of Sec. 6.3).  With UG_F_FUSE half as many again
 * (rounded up): the tail executor runs on a stream of its own for as long
 * as items keep coming, and a stream that shares its hardware queue would
 * wait behind it, so the streams on that queue are set aside when others
 * remain.  Errors: UG_EINVAL. */
ug_status ug_streams_needed(void* ctx, uint32_t* n);

/* Gives the context its stream pool (Sec. 4.4.3: the streams that tasks are
 * bound to).  hip_streams[i] are n distinct HIP streams (hipStream_t) on the
 * context's device, created by the caller at the default priority (e.g.
 * torch.cuda.Stream()); n = ug_streams_needed.  Borrowed: the caller keeps
 * them alive until ug_destroy and issues no work on them meanwhile; the
 * library never destroys them.  The urgency policy takes them as the lanes
 * of level 0, then level 1, ...; FIFO launch as the streams of the chains'
 * tasks in order (register the chains first).  With UG_F_PLACE the order is
 * first rearranged round-robin over the hardware queues the streams use
 * (a probe of about 0.5 ms per stream and queue, synchronous).  Once per
 * context, before ug_start.  Errors: UG_EINVAL (count, null or repeated
 * stream), UG_ESTATE (started, attached before, FIFO without chains),
 * UG_ENODEV, UG_EDEVICE (the probe failed). */
ug_status ug_attach_streams(void* ctx, void* const* hip_streams, uint32_t n);

/* Completed frames (Sec. 6.2: end-to-end latency and deadline miss).
 * Non-blocking: copies up to cap completions into out (caller-owned), oldest
 * first, and removes them from the context.  Returns how many (>= 0), or
 * UG_EDEVICE once a device error has occurred and nothing is left. */
int32_t ug_poll_complete(void* ctx, ug_completion* out, uint32_t cap);

/* Waits up to timeout_ns until every submitted frame has completed
 * (completions stay queued for ug_poll_complete): the end of a run over
 * which Eq. 3 is evaluated.  Errors: UG_ETIMEDOUT, UG_EDEVICE. */
ug_status ug_drain(void* ctx, int64_t timeout_ns);

/* Stops the gate thread after ug_drain and waits for the stream pool to
 * drain; registration stays closed.  The context can be restarted with
 * ug_start (e.g. after ug_set_threshold, Sec. 4.4.3's calibration run
 * followed by the real one).  Errors: UG_EDEVICE. */
ug_status ug_stop(void* ctx);

/* Counters since the last ug_start (submissions, completions, launches,
 * holds, batches, decision instants, time spent deciding and launching):
 * the scheduler-overhead figures of Sec. 6.5.  Errors: UG_EINVAL. */
ug_status ug_get_stats(void* ctx, ug_stats* out);

/* Copies up to cap records of the decision log (every instant's inputs and
 * decisions, for the offline replay of Sec. 4.4's policy) into out and
 * removes them from the log.  Returns how many (>= 0), or UG_EINVAL. */
int32_t ug_trace_read(void* ctx, ug_record* out, uint32_t cap);

/* Copies the calibration samples recorded under UG_F_CALIBRATE (Sec.
 * 4.4.3, the periodically recorded highest urgency among active kernels, as
 * a slack in ns) into out; returns the number copied, UG_EINVAL, or
 * UG_ESTATE while started. */
int32_t ug_calibration_read(void* ctx, int64_t* out, uint32_t cap);

/* TH_urgent from the recorded samples (Sec. 4.4.3): the samples are ordered
 * by urgency (ascending UL = 1/slack) and the nearest-rank pct-th percentile
 * is taken (index ceil(pct/100 * n) - 1).  *th_slack_ns gets its slack, or 0
 * (no task is truly urgent) if that slack is <= 0 or there is no sample.
 * Only while not started. */
ug_status ug_calibration_threshold(void* ctx, int32_t pct, int64_t* th_slack_ns);

/* Deadline metrics over the frames completed since ug_start (Sec. 6.2):
 * Eq. (3) overall miss ratio (mean over chains with completions of
 * missed / completed), and pooled nearest-rank latency percentiles. */
typedef struct {
  uint64_t frames;
  uint64_t missed;
  double miss_ratio;       /* Eq. (3), in [0, 1]                             */
  int64_t p50_ns;
  int64_t p99_ns;
  int64_t max_ns;
  double mean_ns;
  uint32_t n_chains;       /* chains with at least one completed frame       */
  uint32_t pad0;
} ug_metrics;
ug_status ug_get_metrics(void* ctx, ug_metrics* out);

/* Offline replay of one decision instant of Sec. 4.4's policy on a context
 * created with device < 0: applies `inputs` (ARRIVE and EVDONE records) at time t,
 * decides, and writes the decisions to out (COMPLETE..LAUNCH records).
 * *n_out receives their number.  Errors: UG_ESTATE (context has a device),
 * UG_EINVAL (an input the state does not expect), UG_ENOMEM (cap too small). */
ug_status ug_replay_instant(void* ctx, int64_t t, const ug_record* inputs,
                            uint32_t n_inputs, ug_record* out, uint32_t cap,
                            uint32_t* n_out);

/* Launches one kernel directly on a HIP stream (NULL = default stream) with
 * the given buffer pointers, outside any context: a kernel of the lookup
 * table of Sec. 4.1 run in isolation.  Used by the profiling stage and for
 * testing each kernel alone.  The workspace a kernel needs is taken from
 * the device's stream-ordered memory pool.  Asynchronous.  Errors:
 * UG_EINVAL (bad descriptor or missing buffer), UG_EDEVICE. */
ug_status ug_kernel_launch(const ug_kernel* k, void* const* buffers,
                           uint32_t n_buffers, void* hip_stream);

/* Bytes of device workspace a kernel (Sec. 4.1's lookup-table entry) needs
 * beside its buffers (*bytes = 0
 * for most kernels; the voxel scatter of large clouds bins its points
 * through one).  A context allocates the workspace of every registered
 * kernel in ug_chain_register (UG_ENOMEM if that fails); ug_kernel_launch
 * takes a stream-ordered allocation per call.  Errors: UG_EINVAL. */
ug_status ug_kernel_workspace(const ug_kernel* k, uint64_t* bytes);

/* ug_kernel_launch (one kernel of Sec. 4.1 in isolation) with a
 * caller-owned device workspace of workspace_bytes
 * (>= ug_kernel_workspace, 256-byte aligned; may be NULL when that is 0),
 * which must stay untouched until the kernel has finished on hip_stream.
 * It holds no state between launches.  Errors: UG_EINVAL (also: workspace
 * missing, too small or misaligned), UG_EDEVICE. */
ug_status ug_kernel_launch_ws(const ug_kernel* k, void* const* buffers,
                              uint32_t n_buffers, void* workspace,
                              uint64_t workspace_bytes, void* hip_stream);

/* Bytes of the static device workspace of ug_kernel_launch_noalloc, one
 * per GPU the library runs on, held until the process ends. */
#define UG_STATIC_SCRATCH_BYTES (64u << 20)

/* ug_kernel_launch for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): it calls no allocating routine.  A kernel that needs a
 * workspace (ug_kernel_workspace > 0) uses a static device array of
 * UG_STATIC_SCRATCH_BYTES on the current device instead, located on the
 * first call on that device.  The array is shared by every call on that
 * GPU and keeps the last call's contents (no kernel reads what an earlier
 * call left): calls on one stream are ordered, but calls that overlap in
 * time on one GPU (other streams, other threads) race and give wrong
 * results.  Asynchronous.  Errors: UG_EINVAL (bad descriptor or missing
 * buffer; a workspace above UG_STATIC_SCRATCH_BYTES, checked before any
 * device call), UG_EDEVICE. */
ug_status ug_kernel_launch_noalloc(const ug_kernel* k, void* const* buffers,
                                   uint32_t n_buffers, void* hip_stream);

/* Static utilisation of a kernel's launch on `device` (U_k of Sec. 4.1 and
 * Tab. "Example lookup table"): the fraction of the device's compute units
 * its grid occupies, min(1, workgroups / CUs).  Errors: UG_EINVAL,
 * UG_EDEVICE. */
ug_status ug_kernel_util(const ug_kernel* k, int32_t device, float* util);

/* ------------------------------------------------------------------------
 * Fused tails (configuration 2, UG_F_FUSE).  The launch cost that batched
 * launching amortises (Sec. 4.4.5) is, for the short pointwise and reduction
 * kernels after each contraction, most of their time.  The tail executor is
 * one long-lived kernel (one dispatcher and `workers` worker workgroups)
 * that takes such tails from a queue: the host publishes an item with a
 * key, the item becomes ready when its producer's completion counter
 * reaches its target, and the dispatcher hands ready items' tiles (groups of
 * rows) to idle workers smallest key first, so that the most urgent chain's
 * work runs first (Sec. 4.2).  A tail computes y = max(x + b, +0) (the bias+ReLU
 * of UG_OP_BIAS_RELU_F32, bit for bit), then optionally the softmax of each
 * row of y and the sum of each row of y (FP32).  The gate uses it under
 * UG_F_FUSE; the calls below drive it directly.  One thread at a time per
 * queue. */
typedef struct {
  const float* x;          /* X[rows, cols] (device)                         */
  float* y;                /* Y[rows, cols]; may equal x                     */
  const float* bias;       /* b[cols] (axis 0) or b[rows] (axis 1)           */
  float* sm;               /* softmax of the rows of Y [rows, cols]; NULL =
                              none (cols <= 4096 with a softmax)            */
  float* rs;               /* sums of the rows of Y [rows]; NULL = none       */
  uint32_t* counter;       /* the producer's completion counter (device
                              memory, zero before the producer's launch), or
                              NULL: ready at once.  Reset to zero when the
                              item becomes ready.  One producer launch per
                              counter at a time: a counter shared by two
                              outstanding items can leave one never ready  */
  uint32_t counter_target; /* its value once the producer has finished (the
                              *waves of ug_kernel_launch_signal)             */
  uint32_t rows, cols;     /* cols a multiple of 4; x, y, sm and (axis 0)
                              bias 16-byte aligned                          */
  uint32_t axis;           /* 0: bias per column; 1: bias per row           */
} ug_tail;

/* Creates a queue with its executor's stream (default priority), pinned
 * host memory and device memory (allocated here, freed by ug_tails_close).
 * idle_ns: the executor leaves after this long without progress (it is
 * launched again by ug_tails_kick).  log_cap (<= 8192): record the first
 * log_cap tiles served as (publication << 24) | tile.  Errors: UG_EINVAL,
 * UG_EDEVICE. */
ug_status ug_tails_open(int32_t device, uint32_t workers, int64_t idle_ns, uint32_t log_cap,
                        void** queue);
/* Publishes an item with its key (smaller first; ties by slot); returns its
 * slot and publication number.  Its rows per tile: about rows / workers,
 * between 64 KiB and 512 KiB of input (at least one row), rounded up to a
 * multiple of 4.  Errors: UG_EINVAL (shape, alignment, NULL), UG_EAGAIN
 * (all 512 slots hold unfinished items). */
ug_status ug_tails_publish(void* queue, const ug_tail* t, uint64_t key, uint32_t* slot,
                           uint64_t* pub);
/* Rewrites the key of a published item (the gate's re-ranking). */
ug_status ug_tails_set_key(void* queue, uint32_t slot, uint64_t key);
/* Pause: while on, the executor starts no new tile (it still takes in
 * items and keys). */
ug_status ug_tails_pause(void* queue, int32_t on);
/* Launches the executor if items are unfinished and it is not running. */
ug_status ug_tails_kick(void* queue);
/* 1 if the item published as `pub` in `slot` has finished (the slot is
 * free again), 0 if not, < 0 on error. */
int32_t ug_tails_finished(void* queue, uint32_t slot, uint64_t pub);
/* Copies up to cap service-log entries (in the order the tiles were handed
 * to workers); returns the count. */
int32_t ug_tails_log(void* queue, uint64_t* out, uint32_t cap);
/* The executor's statistics as of its last exit (a running executor's
 * current launch is not counted yet), first n of: dispatcher rounds, their
 * total duration, items finished, and over those items the summed time from
 * being taken in to ready (waiting for the producer), from ready to the
 * first tile handed out, and from then to finished, tiles handed out (times
 * in device clock ticks of 10 ns).  Errors: UG_EINVAL, UG_EDEVICE. */
ug_status ug_tails_stats(void* queue, uint64_t* out, uint32_t n);
/* The same statistics for a gate's executor over its last run (from
 * ug_start to ug_stop; read at ug_stop).  Not in ug_stats, whose layout is
 * part of the ABI.  Errors: UG_EINVAL. */
ug_status ug_fuse_stats(void* ctx, uint64_t* out, uint32_t n);
/* Stops the executor, waits for it, frees everything. */
ug_status ug_tails_close(void* queue);

/* ug_kernel_launch with a completion counter: every workgroup of the
 * kernel adds its wavefront count to *counter (device memory, 4-byte
 * aligned) once all its results are stored, with one agent-scope release;
 * *waves receives the total (workgroups x wavefronts per workgroup).  Only UG_OP_GEMM_F32, UG_OP_CONV3X3_F32,
 * UG_OP_GEMM_BF16 and UG_OP_CONV3X3_BF16 take a counter (else UG_EINVAL). */
ug_status ug_kernel_launch_signal(const ug_kernel* k, void* const* buffers,
                                  uint32_t n_buffers, uint32_t* counter, uint32_t* waves,
                                  void* hip_stream);

/* Task graphs (UG_F_GRAPH): captures and instantiates the graph of every
 * task of a chain for one buffer set (buffers as in ug_frame_submit; dims as
 * in ug_frame_submit_dims, or NULL) ahead of the run, so that the gate's
 * first launch of each finds it ready instead of capturing it on the gate
 * thread inside a frame's latency.  With UG_F_FUSE set, the fused variant
 * (tails left out, producers counting) is captured as well.  Before
 * ug_start (the graphs are the gate thread's while it runs); the graphs stay
 * until ug_destroy.  Errors: UG_EINVAL, UG_ESTATE, UG_ENODEV, UG_EDEVICE. */
ug_status ug_graph_prepare(void* ctx, uint32_t chain, void* const* buffers, uint32_t n_buffers,
                           const int64_t* dims, uint32_t n_dims);

/* The raw launch loop of the system-overhead comparison (Sec. 6.5, Tab.
 * "Basic operations"): launches kernel k n times back to back on hip_stream
 * (after 8 untimed launches), then waits.  *host_ns: mean host time per
 * launch call; *gpu_ns: mean device time per kernel over the loop (HIP
 * events around it, so it includes the gaps between kernels).  The cost
 * the gate adds per kernel is set against these.  No workspace kernels
 * (UG_EINVAL).  Synchronous.  Errors: UG_EINVAL, UG_EDEVICE. */
ug_status ug_launch_cost(const ug_kernel* k, void* const* buffers, uint32_t n_buffers,
                         uint32_t n, void* hip_stream, int64_t* host_ns, int64_t* gpu_ns);

/* Tile variants (the autotuner of configuration 2).  The FP32 GEMM has 3
 * tile shapes (0: 128x128, 1: 64x64, 2: 32x32 with a four-way K split) and
 * the FP32 3x3 convolution 5 (output channels x pixel patch, 0: 128 x 8x16,
 * 1: 64 x 8x16, 2: 32 x 8x16, 3: 64 x 2x16 and 4: 32 x 2x16 with a four-way
 * K split); each launcher picks one by a fixed rule unless the process-wide
 * tuning table names one for the exact (op, shape).  Every variant computes
 * the same sums in its own order (results within the op's tolerance, exact
 * for integer-valued inputs).  Set the table before launching (a change is
 * published as a new copy; launches in flight see the old or the new one).
 *   ug_tile_variants   number of variants of an op (0: one tile only)
 *   ug_tile_set        table entry for (op, shape[4]); variant -1 removes it
 *   ug_tile_clear      empty the table
 *   ug_tile_get        the variant a launch of k takes now (-1: one tile)
 *   ug_tile_load       add the entries of a table file: lines
 *                      "op s0 s1 s2 s3 variant", '#' starts a comment;
 *                      *n_added receives the count; a malformed line adds
 *                      nothing (UG_EINVAL)
 *   ug_kernel_launch_variant  ug_kernel_launch at a given variant (timing)
 * Errors: UG_EINVAL. */
int32_t ug_tile_variants(int32_t op);
ug_status ug_tile_set(int32_t op, const int64_t* shape, int32_t variant);
ug_status ug_tile_clear(void);
int32_t ug_tile_get(const ug_kernel* k);
ug_status ug_tile_load(const char* path, uint32_t* n_added);
ug_status ug_kernel_launch_variant(const ug_kernel* k, void* const* buffers, uint32_t n_buffers,
                                   int32_t variant, void* hip_stream);

/* The tails of a registered chain that UG_F_FUSE fuses: (first, end) kernel
 * index ranges (chain-wide numbering), at most cap; returns the count or
 * < 0.  A tail is a bias+ReLU right after a contraction whose output it
 * reads, with at most one row softmax and one row sum of its output after
 * it (same rows and row length); rows a multiple of 4 floats, at most 4096
 * with a softmax; short kernels only (at most 1 MiB of bias+ReLU input: a
 * larger tail gains little from saving launches and runs faster at
 * full-device bandwidth); no per-frame sizes; and no later kernel of the
 * task writes a buffer the tail reads or writes, or reads one it writes (so
 * the tail may run outside the task's stream order). */
int32_t ug_chain_tails(void* ctx, uint32_t chain, int32_t* first, int32_t* end, uint32_t cap);

#ifdef __cplusplus
}
#endif

#endif /* UG_H */
