// Host-side structures of the skeleton runtime: SCT nodes, the linearised
// stage chain, compiled plans and their kernels.
#pragma once
#include <hip/hip_runtime_api.h>

#include <atomic>
#include <string>
#include <vector>

#include "kern.h"
#include "skel.h"

namespace skel {

enum Domain { DOM_NONE = 0, DOM_U8 = 1, DOM_F32 = 2, DOM_NBODY = 3, DOM_C32 = 4, DOM_GRAY = 5 };
enum NodeKind { NK_MAP = 0, NK_PIPE = 1, NK_MAPRED = 2, NK_LOOP = 3, NK_WHILE = 4 };

constexpr int kMaxStages = 4096;       // linearised Map stages after unrolling loops
constexpr int kMaxNBodyIters = 4096;   // N-body loop iterations captured in one graph
constexpr int kMaxDim = 65536;         // image side limit (noise key packs x, y in 16 bits)

// Thread-local error state; set_error returns its status argument.
skel_status set_error(skel_status st, const char* fmt, ...);
void clear_error();

}  // namespace skel

struct skel_node_s {
    std::atomic<int> refs{1};
    int kind = 0;
    int op = -1;
    skel_params prm{};
    std::vector<skel_node_s*> kids;
    int red = -1;
    skel_loop_state loop{};
    skel_loop_cond cond{};
};

namespace skel {

struct Stage {
    int op;            // SKEL_OP_*
    skel_params prm;
    int side_arg;      // SAXPY: argument index of its side vector, else -1
};

// A skeleton tree flattened into depth-first stage order (Sec. 2: the kernels
// of an SCT run sequentially in a depth-first evaluation of the tree).
struct Linear {
    Domain dom = DOM_NONE;
    std::vector<Stage> st;
    int red = -1;                 // SKEL_RED_* or -1
    int nbody_iters = 0;          // Loop(Pipeline(NBODY_FORCE, LEAPFROG)) iterations
    skel_params nbody_prm{};
    uint32_t loop_carried = 0;
    int loop_sync = 0;
    uint32_t seen_ops = 0;        // bit op: stage kind present in the tree (also in 0-trip loops)
    bool is_while = false;        // root is a while Loop over an image MapReduce (st = one iteration)
    int while_max = 0;
    skel_loop_cond wcond{};
    std::string sct;              // textual form of the tree
};

skel_status linearize(skel_node root, Linear& out);

// Resolved configuration (all defaults filled in).
struct Config {
    int fusion = SKEL_FUSE_ON;
    uint32_t split_mask = 0;
    int tile_h = 0;
    int wg = 0;
    int ept = 0;
    int variant = 0;
    bool auto_tile = false;   // tile_h not given: fit each kernel's tiles to one resident round
};

// Compute units of the current device (256 when no device is visible).
int device_cu_count();

// Shape of the arguments a plan is compiled for.
struct Shape {
    int64_t W = 0, H = 0;   // images
    int64_t n = 0;          // vectors
    int64_t N = 0;          // bodies
};

// One kernel of a plan.
struct Kernel {
    int first = 0, last = 0;   // stage range [first, last); empty = reduce-only
    bool blur = false;
    bool reduce = false;
    int src = 0;               // -1 user input, -2 user output, 0/1 scratch image
    int dst = 0;               // -2 user output, 0/1 scratch, -3 none
    ImgGroupArgs img{};        // image kernels (pointers filled per run)
    VecGroupArgs vec{};        // vector kernels
    FftArgs fft{};             // FFT passes (pointers filled per run)
    GrayArgs gray{};           // gray-volume kernels
    int fft_mode = 0;          // 0 pass A, 1 fused B+A, 2 pass B
    std::vector<int> side_args;
    int grid = 0, wg = 0;
    int bins = 256;            // exclusive bound of the values this kernel emits
    const char* name = "";
};

// True when b's strides describe a dense row-major buffer of esize-byte
// elements (all zero, or exactly the dense strides; see plan.cpp).
bool dense_strides(const skel_buffer& b, int64_t esize);
skel_status derive_shape(const Linear& lin, const skel_buffer* proto, int32_t nargs, Shape& sh);
int expected_nargs(const Linear& lin);
skel_status resolve_config(const Linear& lin, const Shape& sh, const skel_plan_opts* opts, Config& cfg);
// Builds the kernel list of (lin, sh, cfg); SKEL_EINVAL if the configuration
// is not valid for this chain (e.g. two stencils forced into one kernel).
skel_status build_kernels(const Linear& lin, const Shape& sh, const Config& cfg, std::vector<Kernel>& ks);
// The partition-validity predicate (Sec. 3.1 constraints, adapted): true when
// the configuration is admissible for this chain and shape.
bool config_valid(const Linear& lin, const Shape& sh, const Config& cfg);

}  // namespace skel

struct skel_plan_s {
    skel_node_s* root = nullptr;
    skel::Linear lin;
    skel::Shape sh;
    skel::Config cfg;
    std::vector<skel_buffer> proto;
    std::vector<skel::Kernel> kernels;
    int device = 0;
    bool resources_ready = false;
    // plan-owned device memory (allocated on the first run)
    void* scratch[2] = {nullptr, nullptr};
    float* partials = nullptr;
    float2* fft_tw = nullptr;       // FFT roots of unity
    uint32_t* hrows = nullptr;      // image reduce: histogram rows, one per work-group
    void* wbuf = nullptr;           // while Loop: second image of the iteration ping-pong
    uint32_t* wstate = nullptr;     // while Loop: device {continue flag, iterations run, previous sum}
    uint32_t* witer_hist = nullptr; // while Loop: one iteration's hist [4][256] when hist is carried ...
    uint64_t* witer_sum = nullptr;  // ... and sums [4] when sum is carried (same allocation)
    uint32_t* h_flag = nullptr;     // while Loop: pinned host copies of the flag, one per block in flight
    hipEvent_t wev[2] = {nullptr, nullptr};  // while Loop: completion of those copies
    float4* nb_acc = nullptr;
    // N-body loop graph
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t gexec = nullptr;
    std::vector<const void*> gkey;
    // batched execution
    skel::BatchReq* d_reqs = nullptr;
    size_t d_reqs_cap = 0;
    uint32_t* d_counter = nullptr;
    skel::BatchReq* h_reqs = nullptr;   // pinned host mirror of the work list
    skel::HistSeg* d_segs = nullptr;    // per-request histogram segments
    skel::HistSeg* h_segs = nullptr;
    uint16_t* d_tile_req = nullptr;     // tile -> request table
    size_t tile_req_cap = 0;
    uint32_t* b_rows = nullptr;         // per-tile histogram rows
    size_t b_rows_cap = 0;              // in words
    hipGraphExec_t bexec = nullptr;
    std::vector<int64_t> bkey;
    int batch_grid = 0;
    // measurement hook (skel_plan_kernel_events)
    int prof_kernel = -1;
    hipEvent_t prof_start = nullptr, prof_end = nullptr;
};

skel_status skel_ensure_resources(skel_plan p);

// Allocation-free runs (skel_plan_run_noalloc): where each scratch buffer of a
// plan sits in one caller-provided device region.
struct NoallocLayout {
    int nimg = 0;
    size_t off_img[2] = {0, 0};
    bool has_partials = false, has_hrows = false;
    size_t off_partials = 0, off_hrows = 0;
    size_t total = 0;
};
// Checks the arguments as skel_plan_run does, then lays out the plan's scratch;
// SKEL_EUNSUPPORTED if the plan needs other resources or more than cap bytes.
skel_status noalloc_prepare(skel_plan p, const skel_buffer* args, int32_t nargs, size_t cap, NoallocLayout& L);
// Enqueues the plan's kernels with its scratch in `region` (device memory of
// at least L.total bytes); the plan's own scratch pointers are left as they were.
skel_status noalloc_run(skel_plan p, const skel_buffer* args, void* stream, char* region, const NoallocLayout& L);

// The host-side checks skel_batch_run makes of a request set (the plan, every
// request on its own, then the requests' buffers against each other), with no
// device work.
skel_status batch_validate(skel_plan p, const skel_buffer* args, int32_t nargs, int32_t nreq);
// Resolves the device address of the static scratch array on `device` (which
// must be current) once; later calls are no-ops.
skel_status noalloc_setup(int device);
