/*
 * hfuse.h -- C ABI of the horizontal-fusion library for AMD gfx950 (MI355X).
 *
 * Horizontal fusion (Sec. I-A, Sec. II-B "Horizontal Kernel Fusion", and the
 * Generate algorithm of Sec. III-A): two independent kernels run as ONE launch.  The threads of a
 * workgroup are cut into two intervals by thread id, [0, d1) and [d1, d1+d2); each
 * interval executes one original kernel body, and each body's workgroup barriers
 * are replaced by barriers that only count the threads of its own interval.  The
 * fused kernel is functionally equivalent to running the two kernels one after
 * the other (Sec. I-A, Sec. III-A "Replace Synchronization Barriers").
 *
 * On CDNA the interval boundary is a multiple of the 64-lane wavefront, the
 * dispatch branch is wave-uniform (no divergence), and the per-interval barrier
 * is an LDS arrival counter (s_barrier always spans the whole workgroup).
 *
 * Conventions shared by every entry point
 *  - All tensor pointers in hf_task are DEVICE pointers on the current HIP device,
 *    owned by the caller.  The library reads hf_task descriptors only during the
 *    call and never frees caller memory.
 *  - `stream` arguments are hipStream_t values passed as void* (NULL = the null
 *    stream).  Work is enqueued and the call returns without synchronising,
 *    unless `ms_out` is non-NULL: then the call records HIP events around the
 *    enqueued work, waits for them and stores the elapsed milliseconds.
 *  - Every function returns HF_OK (0) or a negative hf_status.  Argument errors
 *    (HF_EINVAL / HF_EUNSUPPORTED) are detected on the host before any HIP call,
 *    so they can be exercised without a GPU.  No C++ exception crosses the ABI.
 *  - Scratch: bn_stats and lds_hist keep per-task partial results and arrival
 *    counters in device scratch.  If hf_task.scratch is NULL the library uses
 *    its own arena (one region per concurrently running task of a call,
 *    allocated on first use, zero-filled, released by hf_shutdown).  A caller
 *    may pass its own zero-filled region of hf_scratch_bytes() bytes instead;
 *    every kernel leaves the region zero-filled again when it completes.
 *    Calls that overlap in time on one device and share a scratch region race.
 *  - The library is not thread-safe; it uses the current HIP device.
 */
#ifndef HFUSE_H
#define HFUSE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status codes */
typedef enum {
  HF_OK = 0,
  HF_EINVAL = -1,        /* bad argument: null pointer, shape, split, block, cap, mode */
  HF_EUNSUPPORTED = -2,  /* no compiled instantiation for this (pair, block, cap)       */
  HF_EHIP = -3,          /* a HIP runtime call failed; see hf_last_hip_error()          */
  HF_ETIMEOUT = -4,      /* the watchdog (HF_TIMEOUT_MS) expired while waiting          */
  HF_ENOMEM = -5,        /* device allocation failed                                    */
  HF_ENOMODEL = -6,      /* learned tuner asked for before a model was trained/loaded   */
  HF_ESCRATCH = -7       /* hf_run_fused_noalloc: the tasks' scratch exceeds its static
                            buffer (HF_NOALLOC_SCRATCH_BYTES)                          */
} hf_status;

/* ---------------------------------------------------------------- kernel kinds */
/* The kernel library: the deep-learning kernels of the evaluation (Sec. IV-A,
 * "Benchmark Kernels") that this library implements, plus an integer mixing loop
 * standing in for the compute-bound hash kernels. */
typedef enum {
  HF_BN_STATS = 0,  /* per-channel mean and biased variance of an NCHW fp32 tensor  */
  HF_INT_MIX = 1,   /* R rounds of xorshift(13,17,5) + multiply-add per uint32       */
  HF_IM2COL = 2,    /* image patches -> columns, unfold layout, zero padding         */
  HF_LDS_HIST = 3,  /* 256-bin histogram of uint8 values (bin = byte value)          */
  HF_UPSAMPLE = 4,  /* bilinear upsampling by an integer factor, half-pixel centres  */
  HF_MAXPOOL = 5,   /* 2-D max pooling with the winner's flat index (Sec. IV-A)      */
  HF_SHA256D = 6,   /* SHA-256(SHA-256(header with nonce)), FIPS 180-4               */
  HF_BLAKE2B = 7,   /* BLAKE2b, 32-byte digest, no key, of header with nonce, RFC 7693 */
  HF_ETHASH = 8,    /* Ethash-like: SHA-512 seed, 64 FNV folds of random table rows  */
  HF_NUM_KINDS = 9
} hf_kind;

/* One kernel instance.
 *   kind         hf_kind
 *   in           device input
 *                  BN_STATS, IM2COL, UPSAMPLE,
 *                  MAXPOOL                    : float  [n][c][h][w], contiguous
 *                  INT_MIX                    : uint32 [n]
 *                  LDS_HIST                   : uint8  [n]
 *                  SHA256D, BLAKE2B, ETHASH   : the 80-byte block header; instance
 *                      i hashes header[0:76] || le32(p[0] + i mod 2^32)
 *   out0         device output
 *                  BN_STATS : float mean[c]
 *                  INT_MIX  : uint32 [n]
 *                  IM2COL   : float [n][c*kh*kw][Ho*Wo], Ho=(h+2*pad-kh)/stride+1 (same for Wo)
 *                  LDS_HIST : uint32 counts[256] (overwritten, not accumulated)
 *                  UPSAMPLE : float [n][c][h*s][w*s]
 *                  MAXPOOL  : float [n][c][Ho][Wo], Ho=(h+2*pad-kh)/stride+1 (same for Wo):
 *                             the maximum over the window's in-range elements
 *                  SHA256D, BLAKE2B, ETHASH : uint8 [n][32] digests, 16-byte aligned
 *                             (ETHASH: the eight folded mix words, little-endian)
 *   out1         BN_STATS: float var[c] (biased, divided by n*h*w)
 *                MAXPOOL : int32 [n][c][Ho][Wo] flat index y*w + x, within its
 *                          input plane, of the element each maximum came from
 *                          (row-major scan of the window; a later element wins
 *                          only if greater or NaN, so ties keep the first and
 *                          a NaN propagates), or NULL to skip the indices
 *                unused otherwise
 *   scratch      optional caller scratch (see conventions above), or NULL
 *   n,c,h,w      shape; INT_MIX and LDS_HIST use n as the element count only
 *   p[4]         INT_MIX : p[0] = rounds R >= 0
 *                IM2COL  : p[0]=kh, p[1]=kw, p[2]=stride, p[3]=pad
 *                LDS_HIST: p[0] = number of bins, must be 256
 *                UPSAMPLE: p[0] = integer scale s in [1, 16]
 *                MAXPOOL : p[0]=kh, p[1]=kw, p[2]=stride, p[3]=pad with
 *                          0 <= pad < min(kh, kw) (padded positions never win)
 *                SHA256D, BLAKE2B, ETHASH: p[0] = first nonce (as uint32)
 *   in1          ETHASH: the table, uint32 [h][32] (h rows of 128 bytes,
 *                16-byte aligned, 1 <= h < 2^32); unused (NULL) otherwise.
 *                The seed words s_0..s_15 of a hash are SHA-512 (FIPS 180-4)
 *                of its 80-byte message read as little-endian 32-bit words,
 *                the mix starts as s_(j mod 16), and the row of access j is
 *                fnv(j ^ s_0, mix[j % 32]) % h, with
 *                fnv(a, b) = (a * 16777619) ^ b mod 2^32 (Ethash's access rule).
 * Input and output buffers must be 4-byte aligned (LDS_HIST input: any) and must
 * not overlap.  Element counts must stay below 2^31 per buffer. */
typedef struct {
  int32_t kind;
  int32_t p[4];
  int32_t reserved;
  const void* in;
  void* out0;
  void* out1;
  void* scratch;
  int64_t n, c, h, w;
  const void* in1;
} hf_task;

/* Two independent kernel instances to be fused (K1 and K2 of the Generate
 * algorithm, Sec. III-A). */
typedef struct {
  hf_task a, b;
} hf_pair;

/* A fused-launch configuration.
 *   split_waves  wavefronts of each workgroup given to task a (d1 = 64*split_waves);
 *                the remaining block/64 - split_waves wavefronts run task b.
 *   block        workgroup size d0 in lanes: 256, 512 or 1024.
 *   vgpr_cap     per-lane VGPR bound of the compiled variant (0 = none); one of
 *                0, 64, 80, 96, 128 (Sec. III-B "Limit Register Usage").
 *   grid         workgroups per launch; 0 = occupancy-derived default.       */
typedef struct {
  int32_t split_waves;
  int32_t block;
  int32_t vgpr_cap;
  int32_t grid;
} hf_config;

/* ---------------------------------------------------------------- life cycle */
/* Optional explicit initialisation of the current device (queries properties,
 * creates events).  Every other entry point initialises lazily. */
int hf_init(void);
/* Frees library-owned device memory, events and streams of every device used. */
int hf_shutdown(void);
/* Human-readable text for an hf_status; never NULL. */
const char* hf_strerror(int status);
/* The last hipError_t value recorded by a failing HIP call (0 if none). */
int hf_last_hip_error(void);
/* Library version string. */
const char* hf_version(void);

/* ---------------------------------------------------------------- validation */
/* Host-only checks of one task descriptor: kind, non-null pointers, shapes, p[].
 * Returns HF_OK or HF_EINVAL.  Makes no HIP call. */
int hf_validate_task(const hf_task* t);
/* Bytes of scratch that `t` needs (0 for kinds that need none), or a negative
 * hf_status for an invalid task.  Makes no HIP call. */
int64_t hf_scratch_bytes(const hf_task* t);
/* Host-only check of a fused configuration for a pair (split, block, cap, grid)
 * and of both tasks.  Returns HF_OK, HF_EINVAL or HF_EUNSUPPORTED. */
int hf_validate_fused(const hf_pair* pr, const hf_config* cfg);

/* ---------------------------------------------------------------- execution */
/* One kernel alone (the "original" kernel of the pair), workgroup size `block`
 * (256, 512 or 1024), grid = 0 for the occupancy default.  Its barriers are the
 * native whole-workgroup barrier. */
int hf_run_solo(const hf_task* t, int block, int grid, void* stream, float* ms_out);

enum { HF_SERIAL = 0, HF_STREAMS = 1 };
/* Native baseline (Sec. IV-A "Apply"): the two kernels of the pair launched
 * separately.  HF_SERIAL: a then b, back to back on stream0.  HF_STREAMS: a on
 * stream0 and b on stream1, forked from and joined back into stream0 with events
 * (stream1 may be NULL: the library then uses its own non-blocking stream).  The
 * timed interval runs from before the first launch to after the last kernel
 * ends (Sec. IV-A "Execution Time Measurement"). */
int hf_run_unfused(const hf_pair* pr, int block_a, int block_b, int mode,
                   void* stream0, void* stream1, float* ms_out);

/* The horizontally fused launch (Generate algorithm, Sec. III-A): one kernel, workgroup size
 * `block`, the first split_num/split_den of its lanes run task a and the rest
 * run task b.  split_num*block/split_den must be a positive multiple of 64 that
 * is smaller than block.  vgpr_cap selects the register-bounded variant
 * (0 = unbounded). */
int hf_run_fused(const hf_pair* pr, int split_num, int split_den, int block,
                 int vgpr_cap, void* stream, float* ms_out);
/* Same, with an explicit hf_config (also fixes the grid). */
int hf_run_fused_cfg(const hf_pair* pr, const hf_config* cfg, void* stream,
                     float* ms_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * fused launch as hf_run_fused_cfg, whose tasks without caller scratch get
 * their scratch from a static device array of HF_NOALLOC_SCRATCH_BYTES bytes
 * (one per device, loaded with the library's code object, held until the
 * process ends) instead of the library's allocated arena.  The call makes no
 * allocation on any path (no hipMalloc / hipFree); it enqueues a small kernel
 * that zeroes the scratch regions it uses, then the fused kernel, on `stream`,
 * and returns without waiting (the caller times it with its own events).
 * Returns HF_ESCRATCH, before any HIP call, when the two tasks' regions
 * (hf_scratch_bytes each, rounded up to 256 bytes) exceed the array, e.g.
 * bn_stats over more than about 2^28 elements.  Every call on one device
 * shares that device's array: calls that overlap in time on one device race,
 * so callers on several streams must order them. */
#define HF_NOALLOC_SCRATCH_BYTES (4 << 20)
int hf_run_fused_noalloc(const hf_pair* pr, const hf_config* cfg, void* stream);

/* Vertical fusion, the comparator of Sec. II-B / IV-A: one launch in which
 * every thread of a `block`-lane workgroup runs task a's body and then task b's,
 * each with the native workgroup barrier (grid = 0: occupancy default). */
int hf_run_vfused(const hf_pair* pr, int block, int grid, void* stream, float* ms_out);

/* ---------------------------------------------------------------- resources */
typedef struct {
  int32_t vgprs;          /* VGPRs per lane of the compiled kernel                   */
  int32_t sgprs;          /* reserved, 0: the HIP runtime does not report SGPRs      */
  int32_t lds_bytes;      /* static LDS per workgroup                                */
  int32_t spill_bytes;    /* private (scratch) bytes per lane: register spills       */
  int32_t wg_per_cu;      /* resident workgroups per CU at this block size           */
  int32_t waves_per_simd; /* resident wavefronts per SIMD                            */
  int32_t num_cus;        /* compute units of the device                             */
  int32_t default_grid;   /* grid hf_run_* uses when grid == 0                       */
} hf_kernel_info;
/* Resources of the fused instantiation for (pair kinds, block, cap). */
int hf_fused_info(int kind_a, int kind_b, int block, int vgpr_cap, hf_kernel_info* out);
/* Resources of the solo kernel of `kind` at `block`. */
int hf_solo_info(int kind, int block, hf_kernel_info* out);

/* ---------------------------------------------------------------- tuning */
enum {
  HF_TUNE_EXHAUSTIVE = 0, /* every legal (split, block, cap) of the compiled menu     */
  HF_TUNE_PAPER = 1,      /* Main search of Sec. III-B: d0 = 1024, d1 = 128, 256, ..., 896; each
                             partition profiled without and with the bound r0       */
  HF_TUNE_NAIVE = 2,      /* even split, no bound, no search (Sec. IV-A "Naive")     */
  HF_TUNE_MLP = 3,        /* learned cost model ranks all candidates; only the k
                             best-ranked with pairwise distinct (split, block) are
                             profiled                                               */
  HF_TUNE_EXHAUSTIVE_GRID = 4 /* EXHAUSTIVE, then the launch grid: the three best
                             configurations profiled again at 2, 4 and 8 times the
                             occupancy grid (skipped for a configuration whose
                             default grid is below the occupancy grid).  Beyond the
                             paper, whose fused grid follows the original kernels':
                             every body here is a grid-stride loop, so the grid is
                             free, and a grid larger than the resident workgroups
                             lets a workgroup whose partitions finish at different
                             times leave its CU to the next one                     */
};
typedef struct {
  int32_t n_candidates;   /* candidates the method considered                        */
  int32_t n_profiled;     /* candidates actually launched and timed                  */
  float t_best_ms;        /* median time of the returned configuration               */
  float t_naive_ms;       /* median time of the even split, block 1024, no cap       */
  float wall_s;           /* host wall time of the search                            */
  int32_t reps;           /* timed repetitions per candidate                         */
  int32_t n_solo_launches;/* MLP: solo launches the featurisation made (each kernel at
                             the three block sizes, 6 launches each)                 */
  float solo_ms;          /* MLP: their summed time in milliseconds                  */
} hf_tune_stats;
/* Searches a fused configuration for the pair (Main search, Sec. III-B).  Each
 * profiled candidate is launched `HF_TUNE_REPS` (default 20) times after a warm-up
 * launch; its time is the median.  The choice is the minimum median with the
 * first-found candidate winning ties (the strict comparison of that search).
 * `block` restricts EXHAUSTIVE/EXHAUSTIVE_GRID/MLP to one block size (0 = 256,
 * 512 and 1024).  Only EXHAUSTIVE_GRID returns a nonzero `grid`.
 * Outputs of the pair's tasks are overwritten by the profiling launches. */
int hf_tune(const hf_pair* pr, int method, int block, int topk, void* stream,
            hf_config* best, hf_tune_stats* stats);

/* Median time in milliseconds of `reps` fused launches of `cfg` (after one
 * untimed launch), each bracketed by HIP events on `stream`. */
int hf_profile(const hf_pair* pr, const hf_config* cfg, int reps, void* stream, float* median_ms);

/* Host-only: the candidate configurations `method` considers, in the order it
 * profiles them (before any ranking by the learned model).  vgpr_a, vgpr_b and
 * lds_fused feed the register bound of HF_TUNE_PAPER (ignored otherwise).
 * Writes at most `max` entries to `out` (may be NULL) and returns the total
 * count, or HF_EINVAL. */
int hf_tune_candidates(int method, int block, int vgpr_a, int vgpr_b, int lds_fused,
                       hf_config* out, int max);

/* Register bound r0 of the Main search (Sec. III-B) with gfx950 constants: b_i = R/(d_i*V_i),
 * b0 = min(b1, b2, LDS_CU/LDS(F), T_CU/d0), r0 = R/(b0*d0), R = 131072 lane
 * registers per CU, LDS_CU = 163840 bytes, T_CU = 2048 lanes; all divisions
 * floor.  Inputs are the solo VGPR counts v_a, v_b, the fused kernel's LDS
 * bytes and the partition sizes.  Returns r0 (>= 1) or HF_EINVAL. */
int hf_register_bound(int d1, int d2, int vgpr_a, int vgpr_b, int lds_fused);

/* ---------------------------------------------------------------- learned cost model */
/* A multilayer perceptron (three hidden layers of 64 ReLU units, linear output)
 * that scores fused configurations from HF_MLP_FEATURES features: per kernel
 * (a, then b) a one-hot kind, log2 solo times at blocks 256/512/1024, log2
 * algorithmic bytes and lane-ops, and the fractions of HBM and integer-ALU
 * peak its best solo run reached; then the split fraction, block size, VGPR
 * bound, resident wavefronts per SIMD, three time estimates built from the
 * solo times and the split, the fused instantiation's spill bytes and VGPRs,
 * and the sum of the best solo times.  The tuner trains it on log2(fused time / sum of
 * the best solo times); only the order of its predictions for one pair is
 * used.  Trained and evaluated on the GPU by the library's own kernels.  One
 * model per process, on the device current at hf_mlp_init.  Unless stated
 * otherwise, arrays are HOST pointers, row-major. */
#define HF_MLP_FEATURES 42 /* 2 * (HF_NUM_KINDS + 7) + 10; the last is log2(sum of solo times) */
/* Allocates the model for d_in features: He-uniform weights from `seed`
 * (splitmix64), zero biases, identity feature standardisation. */
int hf_mlp_init(int d_in, uint64_t seed);
/* The same with `members` networks (1..HF_MLP_MAX_MEMBERS), member k drawn
 * from seed + k: hf_mlp_train trains every member on the same data, and
 * predictions are the members' mean (an ensemble, which varies less with the
 * draw of the training pairs than one network).  hf_mlp_get_params,
 * hf_mlp_set_params, hf_mlp_grad, hf_mlp_step and hf_mlp_adam_reset act on
 * the first member. */
#define HF_MLP_MAX_MEMBERS 16
int hf_mlp_init_ensemble(int d_in, uint64_t seed, int members);
/* Members of the current model, or HF_ENOMODEL. */
int hf_mlp_members(void);
/* Number of parameters of the current model, or HF_ENOMODEL. */
int hf_mlp_num_params(void);
/* Copies the flat parameter vector (layout W1[d][64] b1 W2[64][64] b2 W3 b3
 * W4[64][1] b4) out of / into the model; n must equal hf_mlp_num_params(). */
int hf_mlp_get_params(float* host, int64_t n);
int hf_mlp_set_params(const float* host, int64_t n);
/* Mean squared error and its gradient (same layout as the parameters) on
 * already standardised X[n][d], y[n]; parameters are not changed. */
int hf_mlp_grad(const float* X, const float* y, int n, float* loss_out, float* grad_out);
/* One full-batch Adam step (lr, beta1 0.9, beta2 0.999, eps 1e-8) on already
 * standardised data; loss_out (may be NULL) receives the loss before the step. */
int hf_mlp_step(const float* X, const float* y, int n, float lr, float* loss_out);
/* Zeroes Adam's moments and step count. */
int hf_mlp_adam_reset(void);
/* Standardises raw X[n][d] and y[n] with their own mean and deviation (kept in
 * the model), resets Adam and runs `epochs` full-batch steps for every member;
 * loss_out (may be NULL) receives the members' mean standardised training loss
 * after the last step. */
int hf_mlp_train(const float* X, const float* y, int n, int d, int epochs, float lr, float* loss_out);
/* Predictions for raw X[n][d] in the units of the training targets (the mean
 * over the members). */
int hf_mlp_predict(const float* X, int n, float* y_out);
/* Saves / loads the model (parameters and standardisation) to / from a file. */
int hf_mlp_save(const char* path);
int hf_mlp_load(const char* path);
/* Features of `n` fused configurations of the pair.  Runs each task solo at the
 * three block sizes to time it (overwriting the tasks' outputs) on `stream`. */
int hf_featurize(const hf_pair* pr, const hf_config* cfg, int n, void* stream, float* X_out);

/* ---------------------------------------------------------------- batched N-way fusion */
/* Many small instances in ONE persistent launch.  Tasks are cut into groups
 * (group_of_task[i]: nondecreasing ids, each group 1..4 consecutive tasks).
 * Each group runs as an N-way horizontally fused virtual launch: a workgroup of
 * `block` lanes (256, 512 or 1024) gives waves_of_task[i] wavefronts to task i
 * (>= 1 each, at most block/64 per group; NULL = proportional to each task's
 * estimated cost), every task runs its body on its own interval with its own
 * interval barrier, and the persistent workgroups pull (group, virtual
 * workgroup) items from a device queue.  Generalises the two-interval
 * Generate algorithm of Sec. III-A to N intervals.
 * hf_batch_create copies the task table to the device (tasks are read only
 * during the call), allocates scratch for the tasks that need it and have none
 * (zero-filled, left zero-filled by every launch), and returns an opaque handle
 * for the current device.  hf_batch_run launches it on `stream`; with
 * use_graph != 0 the launch is captured once into a HIP graph and the graph is
 * replayed.  Runs of one batch must not overlap in time. */
int hf_batch_create(const hf_task* tasks, int ntask, const int32_t* group_of_task,
                    const int32_t* waves_of_task, int block, void** batch_out);
int hf_batch_run(void* batch, int use_graph, void* stream, float* ms_out);
/* Work items (virtual workgroups summed over groups), persistent grid, groups. */
int hf_batch_info(void* batch, int32_t* total_items, int32_t* grid, int32_t* ngroup);
int hf_batch_destroy(void* batch);
/* create + run + synchronise + destroy. */
int hf_run_batch(const hf_task* tasks, int ntask, const int32_t* group_of_task,
                 const int32_t* waves_of_task, int block, void* stream, float* ms_out);
/* Schedule tuner of a batch: profiles (median of `reps` launches) the cost-
 * proportional and the even wave split at blocks 256, 512 and 1024; writes the
 * best per-task waves (ntask entries) and block, and its median time. */
int hf_batch_tune(const hf_task* tasks, int ntask, const int32_t* group_of_task, int reps, void* stream,
                  int32_t* waves_out, int32_t* block_out, float* ms_out);

/* A batch schedule.
 *   block           workgroup size: 256, 512 or 1024.
 *   interval_waves  0: the static schedule above (each group runs as one N-way
 *                   fused virtual workgroup per work item, intervals sized per
 *                   member, whole-workgroup barriers between items);
 *                   1, 2, 4, 8 or 16 (dividing block/64): worker intervals --
 *                   each workgroup is cut into intervals of this many
 *                   wavefronts, and every interval pulls (task, virtual
 *                   workgroup) items from the device queue on its own, runs
 *                   the task's body on its interval (interval barrier, own LDS
 *                   region) and pulls the next, so the intervals of a
 *                   workgroup run different kernels side by side with no
 *                   whole-workgroup barrier between items.  The queue holds
 *                   the members of each group interleaved item by item, the
 *                   groups in order of decreasing estimated work.
 *   item_kb         estimated traffic of one work item, KiB (0: 256): the
 *                   virtual grid of a task is its traffic over this, capped by
 *                   the workgroups that find work.
 *   split_policy    static schedule without waves_of_task: 0 = wavefronts in
 *                   proportion to each member's estimated cost, 1 = even. */
typedef struct {
  int32_t block;
  int32_t interval_waves;
  int32_t item_kb;
  int32_t split_policy;
} hf_batch_schedule;
/* hf_batch_create under an explicit schedule (waves_of_task must be NULL for
 * worker intervals).  HF_EUNSUPPORTED when the schedule's LDS does not fit a
 * CU (worker intervals with a histogram task need 16 KiB per interval). */
int hf_batch_create_sched(const hf_task* tasks, int ntask, const int32_t* group_of_task,
                          const int32_t* waves_of_task, const hf_batch_schedule* sched, void** batch_out);
/* Schedule search over both kinds of schedule: static (blocks 256/512/1024 x
 * split policy x items of 128/256/512 KiB) and worker intervals (blocks x
 * intervals of 1/2/4/8 wavefronts x items of 64/128/256/512 KiB), every
 * schedule the batch admits profiled as the median of `reps` launches.
 * Writes the fastest schedule, its median time and the number profiled. */
int hf_batch_tune_sched(const hf_task* tasks, int ntask, const int32_t* group_of_task, int reps, void* stream,
                        hf_batch_schedule* best_out, float* ms_out, int32_t* n_profiled);

/* ---------------------------------------------------------------- microbenchmarks */
/* Streams `bytes` (multiple of 16) from src to dst: the reference copy kernel
 * for measured HBM ceilings and for scaling rocprof byte counters. */
int hf_copy(void* dst, const void* src, int64_t bytes, void* stream, float* ms_out);
/* Streams `bytes` (multiple of 16) from src and writes almost nothing: the
 * read-bandwidth ceiling for the reduction kernels. */
int hf_read(const void* src, int64_t bytes, void* stream, float* ms_out);
/* Reads a library-owned 1 GiB buffer (written once, on the first call) so
 * that no input stays in the 256 MB last-level cache between timed
 * repetitions; the lines it leaves behind are clean, so the next kernel pays
 * no write-back for them. */
int hf_scrub(void* stream);
/* Self-test of the interval barrier (the replacement of a counted barrier for
 * one interval of the workgroup, Sec. III-A "Replace Synchronization
 * Barriers"): `grid` workgroups of `block` lanes (0: the resident count), split
 * after `split_waves` wavefronts, run a ring exchange through LDS for iters_a
 * and iters_b rounds, with pseudo-random skew per wavefront and round (from
 * `seed`).  Writes the number of mismatched reads (0 when every barrier held)
 * to the HOST pointer `mismatches`; waits for completion (HF_ETIMEOUT after
 * HF_TIMEOUT_MS). */
int hf_selftest_barrier(int block, int split_waves, int iters_a, int iters_b, uint32_t seed, int grid,
                        void* stream, uint32_t* mismatches);
/* Measured integer-issue ceiling of the int_mix round: `grid` workgroups of 256
 * lanes (0: eight per CU, the resident maximum) each run `rounds` rounds of
 * the round on four independent chains per lane from registers only (the
 * int_mix body's instruction mix without its loads and stores).  Writes the
 * lane-ops executed (8 per lane-round: 3 shifts, 3 xors, 1 multiply, 1 add)
 * to lane_ops_out (may be NULL). */
int hf_int_peak(int rounds, int grid, void* stream, float* ms_out, double* lane_ops_out);
/* Keeps the GPU busy for about `ms` milliseconds (warm-up before measurements,
 * Sec. IV-A "Execution Time Measurement"). */
int hf_warmup(int ms, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* HFUSE_H */
