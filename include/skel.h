/*
 * skel.h -- C-ABI of the MI355X (gfx950) skeleton library.
 *
 * The library executes compound multi-kernel computations on one GPU: Map
 * stages composed into Pipeline, MapReduce and Loop skeletons.  The API
 * mirrors the construction and execution-request constructs of Marrow
 * (arXiv 1510.06585, Sec. 2.1 "The Library" and Table 1): a skeleton
 * computational tree (SCT) is built bottom-up from nodes, compiled once for a
 * set of argument shapes, and then run asynchronously any number of times over
 * caller-owned device buffers.
 *
 * Conventions common to every entry point
 * ---------------------------------------
 * - Every call returns skel_status; SKEL_OK is 0.  On failure a message is
 *   available from skel_last_error() (thread-local, valid until the next call
 *   on the same thread).  No C++ exception crosses this boundary.
 * - Buffers are caller-owned device memory (e.g. from hipMalloc or a PyTorch
 *   tensor).  The library never frees them and never copies them to the host.
 * - Streams and events are passed as `void*` holding a hipStream_t /
 *   hipEvent_t; NULL means the null stream.  Runs are stream-ordered and
 *   asynchronous (the "Future" of Table 1): device-side errors surface at the
 *   next call on that stream or at skel_sync().
 * - Nodes are reference-counted handles released with skel_node_release(); a
 *   node keeps its children alive and a plan keeps its root alive.
 * - A plan owns its scratch memory, kernels and captured graphs and frees them
 *   in skel_plan_destroy().  A plan is used from one host thread at a time;
 *   runs of one plan on different streams must not overlap.
 * - All pointers to host structs may be NULL only where stated.
 */
#ifndef SKEL_H
#define SKEL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status */
typedef int32_t skel_status;
enum {
    SKEL_OK = 0,
    SKEL_EINVAL = 1,        /* bad argument: NULL handle, bad enum, aliasing, count */
    SKEL_ESHAPE = 2,        /* buffer shape or strides do not match the plan       */
    SKEL_ETYPE = 3,         /* dtype mismatch or stages of incompatible domains    */
    SKEL_ENOMEM = 4,        /* device or host allocation failed                    */
    SKEL_EDEVICE = 5,       /* HIP runtime error                                   */
    SKEL_EUNSUPPORTED = 6   /* valid request this library does not implement       */
};

/* ------------------------------------------------------------------ buffers */
/* Data types of vector arguments (the VectorType<T> of Table 1). */
enum { SKEL_U8 = 0, SKEL_U32 = 1, SKEL_U64 = 2, SKEL_F32 = 3, SKEL_F64 = 4 };

/* Buffer flags (Sec. 2.1 immutable arguments; Sec. 3.4 COPY transfer mode). */
#define SKEL_IMMUTABLE 1u   /* the skeleton only reads this buffer                   */
#define SKEL_COPY 2u        /* read whole by every work-group (not partitioned)     */

/* A typed, caller-owned device buffer.  Dense row-major only: over the
 * dimensions of extent > 1, stride_bytes are either all zero (meaning dense)
 * or all equal to the dense strides; anything else, a mix of zero and
 * non-zero strides included, is SKEL_ESHAPE.  Strides of extent-1 dimensions
 * and of buffers with no elements are ignored.  ndim is 1..4. */
typedef struct skel_buffer {
    void* data;
    int32_t dtype;
    int32_t ndim;
    int64_t shape[4];
    int64_t stride_bytes[4];
    uint32_t flags;
    uint32_t reserved;
} skel_buffer;

/* ------------------------------------------------------------ stage set */
/* Built-in Map stages (the leaf kernels of an SCT).  Their arithmetic:
 *  NOISE     (Sec. 4 Filter Pipeline) per pixel (x,y) of the stage's input and
 *            channel byte c: key = seed ^ ((y<<16)|x), h = fmix32(key) (the
 *            MurmurHash3 32-bit finaliser), n = ((h>>8c)&255) mod 33 - 16,
 *            out = clamp(in + n, 0, 255).  Needs W, H <= 65536.
 *  SOLARISE  (Sec. 4) out = in < 128 ? in : 255 - in, every channel byte.
 *  MIRROR    (Sec. 4) left-right within a row: out(x,y) = in(W-1-x,y), whole
 *            pixels; on a 1-D fp32 vector, reversal out[i] = in[n-1-i].
 *  BLUR5     5x5 box blur, floor(window sum / 25), clamp-to-edge addressing.
 *  SAXPY     (Sec. 4 Saxpy) out[i] = fmaf(a, in[i], w[i]); w is this stage's
 *            own side vector (one extra argument per SAXPY stage).
 *  NBODY_FORCE, LEAPFROG (Sec. 4 N-Body) Plummer-softened direct sum
 *            a_i = G sum_j m_j (r_j - r_i) (|r_j - r_i|^2 + eps^2)^(-3/2), then
 *            kick-drift v += dt a, r += dt v.  Only valid as
 *            Pipeline(NBODY_FORCE, LEAPFROG), optionally inside a Loop.
 *  SEGMENT   (Sec. 4 Segmentation) on a gray uint8 volume, every voxel to
 *            black, gray or white: out = v < lo ? 0 : (v < hi ? 128 : 255),
 *            lo <= hi <= 256 (both 0: 85 and 170; lo = hi gives no gray,
 *            hi = 256 no white).  Only SEGMENT stages may share a chain.
 *  FFT, IFFT (Sec. 4 FFT, pipelined with its inversion) per transform of
 *            65536 complex fp32 points (512 KiB): X[k] = sum_n x[n] w^(nk),
 *            w = exp(-2 pi i / 65536) (FFT) or exp(+2 pi i / 65536) with a
 *            1/65536 factor (IFFT).  Only FFT / IFFT stages may share a chain.
 */
enum {
    SKEL_OP_NOISE = 0,
    SKEL_OP_SOLARISE = 1,
    SKEL_OP_MIRROR = 2,
    SKEL_OP_BLUR5 = 3,
    SKEL_OP_SAXPY = 4,
    SKEL_OP_NBODY_FORCE = 5,
    SKEL_OP_LEAPFROG = 6,
    SKEL_OP_FFT = 7,
    SKEL_OP_IFFT = 8,
    SKEL_OP_SEGMENT = 9
};

/* Reduce side of MapReduce (Sec. 2.1; partial results merged by addition,
 * Sec. 3.4).  On RGBA uint8 images:
 *  HIST256_SUM  hist u32 [4][256] (hist[c][v] = #pixels with channel c == v)
 *               and sum u64 [4] (sum of channel c), over the final image.
 *  SUM          sum u64 [4] only.
 * On fp32 vectors only SUM is valid: one f32 scalar, the sum of the final
 * vector (accumulated in fp32 tiles and fp64 across tiles). */
enum { SKEL_RED_HIST256_SUM = 0, SKEL_RED_SUM = 1 };

/* Scalar parameters of a stage (the ScalarType<T> of Table 1).  Fields a
 * stage does not use are ignored. */
typedef struct skel_params {
    uint32_t seed;   /* NOISE */
    float a;         /* SAXPY */
    float eps;       /* NBODY_FORCE softening length */
    float G;         /* NBODY_FORCE gravitational constant */
    float dt;        /* LEAPFROG time step */
    uint32_t lo, hi; /* SEGMENT thresholds (both 0: 85 and 170) */
} skel_params;

/* Loop state (Sec. 2.1: stop condition, items updated per iteration, whether
 * the update needs a global synchronisation).  iterations >= 0 is the count
 * of a counted loop and the limit of a while Loop.  carried_mask: bit k =
 * argument k of the plan is loop state carried from one iteration to the
 * next.  A loop's image, vector or body positions are always carried (each
 * iteration's output feeds the next).  In a while Loop a set bit on a reduce
 * output (hist, sum) makes that output accumulate: every iteration's partial
 * result is merged into it by addition (the merging function of Sec. 3.4),
 * starting from the buffer's content when the run starts; a clear bit leaves
 * the last iteration's result.  Bits beyond the plan's arguments, or on a
 * while Loop's count, are SKEL_EINVAL.  global_sync is recorded and reported
 * by skel_plan_describe; every iteration boundary is a device-wide ordering
 * point regardless. */
typedef struct skel_loop_state {
    int32_t iterations;
    uint32_t carried_mask;
    int32_t global_sync;
} skel_loop_state;

/* Stop condition of a while Loop (Sec. 2.1: Loop covers while loops; the
 * state holds the stoppage condition).  After every iteration i the loop
 * continues while fewer than the state's `iterations` iterations have run and,
 * with s_i the iteration's own uint64 channel sums (before any merge into a
 * carried output),
 *   kind SKEL_COND_VALUE:  s_i[channel] <cmp> threshold
 *   kind SKEL_COND_DELTA:  |s_i[channel] - s_(i-1)[channel]| <cmp> threshold
 *                          (convergence of the reduction; iteration 0 has no
 *                          predecessor and always continues).
 * The condition is evaluated on the device.  check_every > 0: the host
 * enqueues blocks of check_every iterations and, after enqueuing a block,
 * reads the one-word flag left by the block before it to decide whether to
 * enqueue more (a block enqueued after the condition failed does no work);
 * 0 means 8.  check_every < 0: fully asynchronous -- the run enqueues all
 * `iterations` guarded iterations and returns without waiting; iterations
 * after the stop do no work beyond a guard test. */
enum { SKEL_CMP_GT = 0, SKEL_CMP_GE = 1, SKEL_CMP_LT = 2, SKEL_CMP_LE = 3 };
enum { SKEL_COND_VALUE = 0, SKEL_COND_DELTA = 1 };
typedef struct skel_loop_cond {
    int32_t channel;      /* 0..3 */
    int32_t cmp;          /* SKEL_CMP_* */
    uint64_t threshold;
    int32_t check_every;  /* > 0: iterations between host checks; 0 = 8; < 0 = no host checks */
    int32_t kind;         /* SKEL_COND_VALUE or SKEL_COND_DELTA */
} skel_loop_cond;

/* -------------------------------------------------------- plan options */
enum { SKEL_FUSE_AUTO = -1, SKEL_FUSE_OFF = 0, SKEL_FUSE_ON = 1, SKEL_FUSE_MASK = 2 };
enum { SKEL_SELECT_DEFAULT = 0, SKEL_SELECT_DB = 1, SKEL_SELECT_MODEL = 2, SKEL_SELECT_EXHAUSTIVE = 3 };

/* Execution configuration of a plan (the per-SCT framework configuration the
 * paper's Auto Tuner and Knowledge Base produce, Sec. 2.2 and Sec. 3.2).
 * Zero in tile_h / wg / ept means "default".
 *  fusion      SKEL_FUSE_ON: fuse every legal run of adjacent stages (at most
 *              one stencil per kernel); OFF: one kernel per stage, the
 *              depth-first plain execution of Sec. 2; MASK: split_mask bit i
 *              set = start a new kernel after stage i, and bit (k-1) for a
 *              k-stage chain = run the reduce side as its own kernel.
 *  tile_h      rows one wavefront sweeps per image tile (image stages), or
 *              j-slices per body group (N-body).
 *  wg          work-group size in threads (multiple of 64, <= 1024).
 *  ept         16-byte vectors per thread per row (fp32 chains: per thread).
 *  variant     0: a kernel specialised for the stage chain when one exists,
 *              1: always the generic stage interpreter (image chains); for an
 *              N-body Loop, launch the iterations one by one instead of
 *              replaying a captured graph.
 *  select      how skel_plan_compile fills fields left at their defaults
 *              (DEFAULT = built-in defaults; the others are used by
 *              skel_tune / skel_cost_select, which return explicit options). */
typedef struct skel_plan_opts {
    int32_t fusion;
    uint32_t split_mask;
    int32_t tile_w;
    int32_t tile_h;
    int32_t wg;
    int32_t ept;
    int32_t select;
    int32_t variant;
} skel_plan_opts;

typedef struct skel_node_s* skel_node;
typedef struct skel_plan_s* skel_plan;

/* Fills *opts with the defaults (fusion ON, everything else 0). */
void skel_plan_opts_default(skel_plan_opts* opts);

/* Binds the calling host thread to HIP device `device` and checks it is a
 * gfx950 part.  Optional: other calls use the current device. */
skel_status skel_init(int32_t device);

/* ------------------------------------------------------ SCT construction */
/* Map(Kernel): a leaf stage `op` (SKEL_OP_*) with scalars *p (may be NULL:
 * all zero).  Table 1 "map" / "kernel". */
skel_status skel_map(int32_t op, const skel_params* p, skel_node* out);

/* Pipeline(SCT... stages): n >= 1 control- and data-dependent stages run in
 * order, stage k's output feeding stage k+1 (Table 1 "pipeline").  The new
 * node holds references to the stages; the caller keeps its own. */
skel_status skel_pipeline(const skel_node* stages, int32_t n, skel_node* out);

/* MapReduce(map, reduce): map followed by the reduce side `red`
 * (SKEL_RED_*), Table 1 "map_reduce".  Valid only at the root of a plan. */
skel_status skel_mapreduce(skel_node map, int32_t red, skel_node* out);

/* Loop(body, state): runs `body` st->iterations times, each iteration's
 * output feeding the next (Table 1 "loop").  Loops over image or vector
 * stages unroll into the stage chain (depth-first order, Sec. 2); a loop over
 * Pipeline(NBODY_FORCE, LEAPFROG) keeps its state on the device and is
 * captured into one HIP graph. */
skel_status skel_loop(skel_node body, const skel_loop_state* st, skel_node* out);

/* While Loop(body, state, cond) with a device-evaluated stop condition (the
 * paper evaluates a Loop's condition and updates its state on the host,
 * Sec. 3.1; here both stay on the device).  body must be a MapReduce over an
 * image chain (SKEL_RED_HIST256_SUM or SKEL_RED_SUM); st->iterations >= 1 is
 * the iteration limit.  Valid only at the root of a plan.  A run computes
 *     x = in; count = 0; H = hist; S = sum;           (caller's initial state)
 *     do { (x, h, s) = body(x); ++count;
 *          H = carried(hist) ? H + h : h;  S = carried(sum) ? S + s : s; }
 *     while (count < st->iterations && cond(s));
 * and writes out = x, hist = H, sum = S and count (uint32 counters and uint64
 * sums wrap).  Plan arguments: in u8 [H,W,4], out u8 [H,W,4],
 * [hist u32 [4,256],] sum u64 [4], count u32 [1]; no two may overlap.  With
 * cond->check_every >= 0 a run blocks the host: after enqueuing each block of
 * check_every iterations it waits for the previous block to finish; with
 * check_every < 0 it is asynchronous like every other run.  Errors:
 * SKEL_EINVAL for a bad channel, cmp, kind, limit or carried_mask bit. */
skel_status skel_loop_while(skel_node body, const skel_loop_state* st, const skel_loop_cond* cond,
                            skel_node* out);

/* Drops one reference; frees the node when none remain. NULL is a no-op. */
skel_status skel_node_release(skel_node node);

/* ------------------------------------------------------ plans */
/* Compiles `root` for arguments shaped like proto[0..nargs) (only dtype, ndim
 * and shape are read; data may be NULL).  Argument order:
 *  image chains   in u8 [H,W,4], out u8 [H,W,4]
 *                 [, hist u32 [4,256], sum u64 [4]]   (HIST256_SUM)
 *                 [, sum u64 [4]]                     (SUM)
 *  fp32 chains    in f32 [n], one side f32 [n] per SAXPY stage, out f32 [n]
 *                 [, sum f32 [1]]                     (SUM)
 *  N-body         pos f32 [N,4] (x,y,z,m), vel f32 [N,4] (w unused),
 *                 pos_scratch f32 [N,4]; after a run the positions are in pos.
 *  gray chains    in u8 [D,H,W] (any 1..4-D shape, fewer than 2^31 voxels),
 *                 out u8 of the same shape; in == out is allowed (voxel-wise
 *                 stages), any other overlap is rejected
 *  FFT chains     in f32 [B,65536,2], out f32 [B,65536,2] (B transforms,
 *                 interleaved re, im; in and out must not overlap).  A fused
 *                 chain of L stages runs L + 1 kernels (the second half of
 *                 a stage and the first half of the next share one), an
 *                 unfused one 2L; split_mask bits split between stages.
 * opts may be NULL (defaults).  Compilation is host-only: the plan's device
 * scratch (intermediate images between unfused kernels, partial sums, graph
 * state) is allocated on the current device by its first run.  Errors:
 * SKEL_ETYPE (mixed stage domains), SKEL_ESHAPE, SKEL_EINVAL (invalid
 * options), SKEL_EUNSUPPORTED (e.g. W or H > 65536, an image over 2 GiB). */
skel_status skel_plan_compile(skel_node root, const skel_buffer* proto, int32_t nargs,
                              const skel_plan_opts* opts, skel_plan* out);

/* Execution request (Table 1 "run"): enqueues the plan on `stream` over args
 * shaped exactly like the prototypes.  Reduce outputs are overwritten (not
 * accumulated).  In-place use (in == out) is SKEL_EINVAL when the kernel that
 * reads the input and writes the output contains a stencil or a mirror.  The
 * first run allocates the plan's device scratch (SKEL_ENOMEM on failure) and,
 * for an N-body Loop, captures its HIP graph; later runs allocate nothing.
 * The buffers and the plan must stay alive until the work completes. */
skel_status skel_plan_run(skel_plan plan, const skel_buffer* args, int32_t nargs, void* stream);

/* As skel_plan_run, then records hipEvent_t `done` on the stream (the
 * paper's Future).  done may be NULL. */
skel_status skel_plan_run_event(skel_plan plan, const skel_buffer* args, int32_t nargs,
                                void* stream, void* done);

/* Batched execution of many requests over distinct data sets in content and
 * size (Sec. 2, batch execution model): args[r*nargs + k] is argument k of
 * request r, each request shaped like an image-chain plan's arguments but
 * with its own H and W (<= 65536).  All requests run in one persistent
 * kernel fed by a work list (largest requests first), captured into a HIP
 * graph that is replayed while the same buffers and shapes are passed again.
 * The plan must be a single-kernel (fully fused) image chain.  Within a
 * request in == out is allowed only for chains without a stencil or mirror;
 * any other overlap of a written buffer (out, hist, sum) with a buffer of the
 * same or another request is SKEL_EINVAL (inputs may be shared). */
skel_status skel_batch_run(skel_plan plan, const skel_buffer* args, int32_t nargs,
                           int32_t nreq, void* stream);

/* Allocation-free execution request, for callers that cannot allocate device
 * memory while they run (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, checks, ordering and
 * results as skel_plan_run, but the plan's device scratch (intermediate
 * images / vectors / volumes of unfused plans, fp32 reduce partials, image
 * histogram rows) is carved out of one static device array of
 * SKEL_NOALLOC_SCRATCH_BYTES per GPU, which the library holds from module
 * load until the process ends; the call itself never allocates (no hipMalloc,
 * hipFree or host allocation).  Covers image chains (not while Loops), fp32
 * chains and gray chains; N-body Loops, FFT chains and while Loops are
 * SKEL_EUNSUPPORTED, and so is a plan whose scratch exceeds the array
 * (every fused image chain up to the 2 GiB image limit fits; unfused plans
 * need two intermediate images).  Every call on one GPU shares that GPU's
 * array and leaves its contents behind: calls that overlap in time on one GPU
 * (different streams, or different host threads) race and must be ordered by
 * the caller, e.g. by using one stream.  The device address of the array is
 * looked up by skel_init(device), or by this call's first use on a device. */
#define SKEL_NOALLOC_SCRATCH_BYTES (32u << 20)
skel_status skel_plan_run_noalloc(skel_plan plan, const skel_buffer* args, int32_t nargs, void* stream);

/* Writes a one-line JSON description (linearised stages, kernels and their
 * stages, configuration) into buf (NUL-terminated, truncated to len). */
skel_status skel_plan_describe(skel_plan plan, char* buf, size_t len);

/* Measurement hook: while set, every run of the plan records hipEvent_t
 * `start` and `end` around kernel `kernel` (an index into the kernels
 * skel_plan_describe lists), so the kernel's own duration can be read with
 * hipEventElapsedTime.  Image kernels take both timestamps from their own
 * dispatch (hipExtLaunchKernel), which brackets the kernel's execution
 * exactly; other kernels have the events recorded on the stream immediately
 * before and after the launch.  kernel < 0 or NULL events clear the hook.  Not
 * applied inside captured graphs (N-body loops, batched runs).  The caller
 * owns the events. */
skel_status skel_plan_kernel_events(skel_plan plan, int32_t kernel, void* start, void* end);

/* Frees the plan and everything it owns; waits for none of its work (the
 * caller synchronises first).  NULL is a no-op. */
skel_status skel_plan_destroy(skel_plan plan);

/* Waits for `stream` and reports any pending device error. */
skel_status skel_sync(void* stream);

/* Message of the last failing call on this thread ("" if none). */
const char* skel_last_error(void);

/* ------------------------------------------- auto-tuning and cost model */
/* Auto Tuner (Sec. 2.2; search in the spirit of Algorithm 1): times the
 * valid configurations of `root` over the given (device) arguments -- fusion
 * partition x work-group size x vectors per thread x tile height, filtered
 * by the partitioning constraints of Sec. 3.1 -- with 3 warm-up runs and the
 * median of `reps` timed runs each (reps <= 0: 10).  max_configs <= 0 times
 * every configuration (exhaustive); otherwise a sample of that many, drawn
 * with `sample_seed`, always including the default configuration.  Appends
 * one row per timed configuration to the text database `db_path` (may be
 * NULL): key, fusion, split_mask, tile_h, wg, ept, variant, the 24 cost-model
 * features, median and minimum microseconds.  Writes the fastest
 * configuration to *best and its median time to *best_us (may be NULL).
 * Synchronises the device; the arguments' contents are overwritten. */
skel_status skel_tune(skel_node root, const skel_buffer* args, int32_t nargs, const char* db_path,
                      int32_t reps, int32_t max_configs, uint64_t sample_seed, skel_plan_opts* best,
                      double* best_us);

/* Profile building by Algorithm 1 (Sec. 3.2), on one GPU: the candidate set
 * of skel_tune is walked as ordered dimensions with early stopping instead of
 * exhaustively.  Fusion partitions go fewest kernels first, and the search
 * ends at the first partition (after the first) that does not improve on the
 * best time; per partition, work-group sizes go in non-increasing order of
 * occupancy (resident wavefronts per CU; sizes below occ_threshold x the best
 * occupancy are filtered out, 0 keeps all), and the first size that does not
 * improve ends that partition; per size, the inner parameter (image tile
 * height, fp32 vectors per thread, N-body j-slices) increases while each step
 * improves by at least precision_us microseconds.  Every timed configuration
 * is appended to db_path (may be NULL) in skel_tune's format; *timed (may be
 * NULL) receives their number.  Timing, synchronisation and the overwriting
 * of the arguments are as in skel_tune. */
skel_status skel_tune_pruned(skel_node root, const skel_buffer* args, int32_t nargs, const char* db_path,
                             int32_t reps, double precision_us, double occ_threshold, skel_plan_opts* best,
                             double* best_us, int32_t* timed);

/* Times one configuration of `root` over the given (device) arguments with
 * the tuner's protocol (a fresh plan compiled with *opts -- NULL: defaults --,
 * 3 warm-up runs, then `reps` runs each bracketed by HIP events on a private
 * stream; reps <= 0: 10), so that a baseline or a re-timing compares with the
 * tuning database's rows like for like.  Writes the median and (may be NULL)
 * minimum in microseconds.  Synchronises the device; the arguments' contents
 * are overwritten.  Compile errors are reported as by skel_plan_compile. */
skel_status skel_time_config(skel_node root, const skel_buffer* args, int32_t nargs, const skel_plan_opts* opts,
                             int32_t reps, double* median_us, double* min_us);

/* Auto Tuner for batched runs (Sec. 2.2 applied to the batch execution
 * model of Sec. 2): times skel_batch_run of the request set args[r*nargs+k]
 * (nreq requests shaped as for skel_batch_run) over tile height x work-group
 * size of the fully fused plan of `root` (the only partition a persistent
 * batched launch holds): tile heights {8, 12, 16, 24, 31, 40, 48, 64, 96,
 * 128} rows x work-groups of {64, 128, 256} threads (1, 2 or 4 adjacent
 * tiles per group), each with 3 warm-up runs and the median of `reps` timed
 * runs (reps <= 0: 10).  pruned == 0 times every point; otherwise the walk of
 * Algorithm 1: sizes in non-increasing order of resident wavefronts per CU,
 * stopping at the first size that does not improve, and per size tile
 * heights increasing while each improves by at least precision_us.  Appends
 * one row per timed point to db_path (may be NULL) in skel_tune's format,
 * after a provenance line; the key starts with "batch<nreq>|px<pixels>|" and
 * the features describe a square image of the batch's total pixel count.
 * Writes the fastest options to *best (fusion ON, tile_h, wg), its median to
 * *best_us and the number of points timed to *timed (both may be NULL).
 * Before any device work the request set gets skel_batch_run's host-side
 * checks, so a bad request returns that call's status and message (EINVAL,
 * ESHAPE, EUNSUPPORTED); a candidate that fails to run afterwards is
 * SKEL_EDEVICE.  Synchronises the device; the requests' outputs are
 * overwritten. */
skel_status skel_tune_batch(skel_node root, const skel_buffer* args, int32_t nargs, int32_t nreq,
                            const char* db_path, int32_t reps, int32_t pruned, double precision_us,
                            skel_plan_opts* best, double* best_us, int32_t* timed);

/* Number of valid configurations skel_tune would time exhaustively for
 * (root, shapes), i.e. the cost model's candidate set. */
skel_status skel_config_count(skel_node root, const skel_buffer* proto, int32_t nargs, int32_t* count);

/* Number of features of the cost model (24) and the feature vector of
 * (root, shapes, opts).  feat must hold skel_feature_count() floats. */
int32_t skel_feature_count(void);
skel_status skel_features(skel_node root, const skel_buffer* proto, int32_t nargs,
                          const skel_plan_opts* opts, float* feat);

/* Cost-model MLP 24 -> 64 -> 64 -> 1 (ReLU), fp32, on the GPU.  Replaces the
 * paper's configuration derivation by interpolation (Sec. 3.2).  Parameters
 * are 5825 floats, W1 [64,24] row-major, b1 [64], W2 [64,64], b2 [64],
 * W3 [1,64], b3 [1].  All pointers are device pointers.
 *  forward   y[i] = MLP(X[i,:]) for X f32 [n,24].
 *  grad      *loss = mean_i (y_i - t_i)^2 and grad f32 [5825] = dloss/dparams.
 *  adam      one Adam step (bias-corrected, step counts from 1) in place on
 *            params, m, v given grad. */
int32_t skel_mlp_param_count(void);
skel_status skel_mlp_forward(const float* params, const float* X, int32_t n, float* y, void* stream);
skel_status skel_mlp_grad(const float* params, const float* X, const float* t, int32_t n,
                          float* grad, float* loss, void* stream);
skel_status skel_mlp_adam(float* params, const float* grad, float* m, float* v, int32_t step,
                          float lr, float beta1, float beta2, float eps, void* stream);

/* Trains the cost model on the rows of `db_path` (log-runtime targets) for
 * `epochs` epochs of mini-batch Adam on the GPU, starting from the host
 * initial parameters init (5825 floats; NULL = He-uniform from `seed`),
 * shuffling with `seed`; writes the trained parameters to `weights_out` (text)
 * and the final mean training loss to *final_loss (may be NULL). */
skel_status skel_cost_train(const char* db_path, const char* weights_out, int32_t epochs,
                            uint64_t seed, const float* init, float* final_loss);

/* Scores every valid configuration of (root, shapes) with the trained model
 * in `weights` (one GPU forward pass over all candidates) and writes the one
 * with the lowest predicted runtime to *chosen.  `weights` may list several
 * model files separated by ';' (an ensemble): their log-runtime predictions
 * are averaged (also for skel_cost_rank). */
skel_status skel_cost_select(skel_node root, const skel_buffer* proto, int32_t nargs,
                             const char* weights, skel_plan_opts* chosen);

/* The model as a shortlist for the profiler (the derivation of Sec. 3.2
 * narrowing what Algorithm 1 has to time): writes the min(k, #valid)
 * configurations with the lowest predicted runtime to ranked[0..*count), in
 * increasing predicted time (ranked[0] is skel_cost_select's choice), and the
 * predicted times in microseconds to pred_us (may be NULL).  ranked and
 * pred_us are caller-owned arrays of at least k entries; k >= 1. */
skel_status skel_cost_rank(skel_node root, const skel_buffer* proto, int32_t nargs, const char* weights,
                           int32_t k, skel_plan_opts* ranked, float* pred_us, int32_t* count);

#ifdef __cplusplus
}
#endif
#endif /* SKEL_H */
