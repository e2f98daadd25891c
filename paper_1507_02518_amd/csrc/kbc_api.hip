// kbc_api.hip -- C-ABI of the D3Q27 KBC box (declared in include/kbc.h):
// argument checking, device memory, the step counter and layout bookkeeping,
// diagnostics read-back and error reporting.  Every computation on the
// populations runs in the kernels of kbc_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "kbc.h"
#include "kbc_internal.h"

using namespace kbc;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg)
{
    g_last_error = msg;
    return code;
}

int hip_fail(hipError_t e, const char* where)
{
    if (e == hipErrorOutOfMemory) return fail(KBC_ENOMEM, std::string(where) + ": out of device memory");
    return fail(KBC_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

#define KBC_HIP(call)                                         \
    do {                                                      \
        hipError_t e_ = (call);                               \
        if (e_ != hipSuccess) return hip_fail(e_, #call);     \
    } while (0)

size_t elem_bytes(int dtype)
{
    return dtype == KBC_F64 ? 8 : (dtype == KBC_F16_DEV ? 2 : 4);
}

// Gap between consecutive direction planes.  When the plane size is a
// multiple of 64 MiB and large, the 27 read and 27 write streams of a sweep
// start at addresses that agree in all the low bits, and on MI355X they then
// contend for the same HBM channels and banks: a 512^3 box ran 10% (FP64 AA),
// 2% (FP64 pull), 21% (FP32 AA) and 11% (FP16 AA, 256 MiB planes) slower
// than with the planes offset by 4352 bytes (17 x 256).  For smaller planes
// the same offset cost 4-17% (FP32 AA at 64 MiB, FP64 AA at 128 MiB), and
// for an FP32 pull sweep at 512 MiB planes 1%, so the gap is applied only
// where it was measured to help.
constexpr uint64_t kPlaneGapBytes = 4352;

uint64_t plane_pad_elems(uint64_t nnodes, size_t elem, int streaming)
{
    const uint64_t bytes = nnodes * elem;
    const bool aligned = bytes % (64ull << 20) == 0;
    const uint64_t from = streaming == KBC_AA ? (256ull << 20) : (1024ull << 20);
    if (!aligned || bytes < from) return 0;
    return kPlaneGapBytes / elem;
}

}  // namespace

void kbc::set_last_error(const char* msg) { g_last_error = msg ? msg : ""; }

struct kbc_box {
    int64_t shape[3];
    Geom g;
    int dtype, variant, streaming;
    bool exact_gamma;   // root of Eq. result1 instead of the estimate
    Coll coll;
    double nu;
    int device;
    hipStream_t stream;
    bool own_stream;
    void* buf[2];       // pull: two lattices; AA: buf[0] only
    int cur;            // pull: buffer holding P(t-1)
    int64_t t;
    float scale[27], inv_scale[27];
    int8_t scale_exp[28];   // the same scales as powers of two, for the step kernels
    bool scales_set;
    bool initialised;
    bool xcd_eighths;  // AA sweeps with one eighth of the workgroups per XCD (step_block)
    // diagnostics scratch (allocated on first use)
    double* d_u;
    double* d_rho;
    double* d_partial;
    double* d_sum;      // [0..2] mean sums, [3..5] second reduction, [8..15]
                        // gradient statistics, [16..19] gamma statistics
    int* d_flag;
    unsigned* d_max;
    double* d_pop;      // canonical staging [27][N]
    // kStepGraph consecutive steps as one graph, built on first use, for the
    // state it starts from (pull: P(t-1) in buf[0]; AA: even t); its kernel
    // arguments hold the buffers, geometry, constants and FP16 exponents, so
    // it is dropped whenever the exponents change
    hipGraph_t graph;
    hipGraphExec_t graph_exec;
};

namespace {

int check_handle(kbc_handle h)
{
    if (!h) return fail(KBC_EINVAL, "null handle");
    return KBC_OK;
}

int set_device(kbc_handle h)
{
    KBC_HIP(hipSetDevice(h->device));
    return KBC_OK;
}

int layout_now(const kbc_box* h)
{
    if (h->streaming == KBC_PULL) return LY_PULL;
    return (h->t % 2 == 0) ? LY_AA_EVEN : LY_AA_ODD;
}

void* state_buf(const kbc_box* h)
{
    return h->streaming == KBC_PULL ? h->buf[h->cur] : h->buf[0];
}

// The small device buffers of a box (a few KB): reduction partials and
// sums, the non-finite flag, the FP16 maxima.
int ensure_small(kbc_handle h)
{
    if (!h->d_partial) KBC_HIP(hipMalloc(&h->d_partial, 8 * (size_t)reduce_partials() * sizeof(double)));
    if (!h->d_sum) KBC_HIP(hipMalloc(&h->d_sum, 32 * sizeof(double)));
    if (!h->d_flag) KBC_HIP(hipMalloc(&h->d_flag, sizeof(int)));
    if (!h->d_max) KBC_HIP(hipMalloc(&h->d_max, 27 * sizeof(unsigned)));
    return KBC_OK;
}

// The large buffers are allocated on first use, so that a box that is only
// initialised from device memory and stepped holds its populations and the
// small buffers alone: the velocity field the diagnostics reduce over (24 B
// per node), the density when asked for (8 B per node), the FP64 population
// copy of get / set populations (216 B per node).
int ensure_diag(kbc_handle h, bool need_rho)
{
    if (int r = ensure_small(h)) return r;
    const size_t N = h->g.nnodes;
    if (!h->d_u) KBC_HIP(hipMalloc(&h->d_u, 3 * N * sizeof(double)));
    if (need_rho && !h->d_rho) KBC_HIP(hipMalloc(&h->d_rho, N * sizeof(double)));
    return KBC_OK;
}

int ensure_pop(kbc_handle h)
{
    if (int r = ensure_small(h)) return r;
    if (!h->d_pop) KBC_HIP(hipMalloc(&h->d_pop, 27 * (size_t)h->g.nnodes * sizeof(double)));
    return KBC_OK;
}

// FP16 scales: a power of two per direction so that the largest deviation
// maps to about 2^12, equal for opposite directions.
void choose_scales(kbc_handle h, const unsigned* max_bits)
{
    for (int i = 0; i < 27; ++i) {
        float m0, m1;
        std::memcpy(&m0, &max_bits[i], sizeof(float));
        std::memcpy(&m1, &max_bits[26 - i], sizeof(float));
        double m = std::max<double>(m0, m1);
        m = std::max(m, 1e-4 * weight(i));
        // within the int8 range, and defined for a non-finite maximum
        const int e = (int)std::min(126.0, std::max(-126.0, std::floor(std::log2(4096.0 / m))));
        h->scale[i] = std::ldexp(1.0f, e);
        h->inv_scale[i] = std::ldexp(1.0f, -e);
        h->scale_exp[i] = (int8_t)e;
    }
    h->scales_set = true;
}

// Moments of the current state into h->d_u / h->d_rho; returns KBC_EUNSTABLE
// when a value is not finite.
int compute_moments(kbc_handle h, bool want_rho)
{
    int r = ensure_diag(h, want_rho);
    if (r) return r;
    KBC_HIP(hipMemsetAsync(h->d_flag, 0, sizeof(int), h->stream));
    KBC_HIP(launch_moments(h->dtype, layout_now(h), state_buf(h), h->g, h->inv_scale,
                           want_rho ? h->d_rho : nullptr, h->d_u, h->d_flag, h->stream));
    int flag = 0;
    KBC_HIP(hipMemcpyAsync(&flag, h->d_flag, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    KBC_HIP(hipStreamSynchronize(h->stream));
    if (flag) return fail(KBC_EUNSTABLE, "state is not finite (the run has diverged)");
    return KBC_OK;
}

// Steps per graph of kbc_step (0: every step is its own launch).  A box
// advanced n >= kStepGraph steps replays the graph floor(n / kStepGraph)
// times after at most one single step that brings it to the graph's start
// state; the remainder runs as single launches.  The graph holds the same
// kernels with the same arguments as the single launches, so the results
// are the same bits.
#ifndef KBC_STEP_GRAPH
#define KBC_STEP_GRAPH 16
#endif
constexpr int kStepGraph = KBC_STEP_GRAPH;
static_assert(kStepGraph % 2 == 0, "a graph must return the box to its start state");

void drop_graph(kbc_handle h)
{
    if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    h->graph_exec = nullptr;
    h->graph = nullptr;
}

bool at_graph_start(const kbc_box* h)
{
    return h->streaming == KBC_PULL ? h->cur == 0 : h->t % 2 == 0;
}

StepParams step_params(const kbc_box* h)
{
    StepParams p;
    std::memset(&p, 0, sizeof(p));
    p.g = h->g;
    p.c = h->coll;
    static_assert(sizeof(p.scale_exp) == sizeof(h->scale_exp), "exponent layout");
    std::memcpy(p.scale_exp, h->scale_exp, sizeof(p.scale_exp));
    p.xcd_order = h->xcd_eighths ? ORDER_EIGHTHS : ORDER_PAIRS;
    return p;
}

// Sweep and buffers of the step taken from pull buffer `cur` or AA time t.
int step_sweep(const kbc_box* h, int cur, int64_t t, StepParams& p)
{
    if (h->streaming == KBC_PULL) {
        p.src = h->buf[cur];
        p.dst = h->buf[1 - cur];
        return SW_PULL;
    }
    p.src = h->buf[0];
    p.dst = h->buf[0];
    return t % 2 == 0 ? SW_AA_EVEN : SW_AA_ODD;
}

int build_graph(kbc_handle h)
{
    hipGraph_t graph = nullptr;
    KBC_HIP(hipGraphCreate(&graph, 0));
    StepParams p = step_params(h);
    hipGraphNode_t prev = nullptr;
    hipError_t e = hipSuccess;
    for (int k = 0; k < kStepGraph && e == hipSuccess; ++k) {
        const int sweep = step_sweep(h, k % 2, k, p);
        StepFn fn;
        uint32_t grid, block;
        e = step_launch_shape(h->dtype, h->variant, sweep, h->exact_gamma, h->g, &fn, &grid, &block);
        if (e != hipSuccess) break;
        void* args[] = {&p};
        hipKernelNodeParams np;
        std::memset(&np, 0, sizeof(np));
        np.func = reinterpret_cast<void*>(fn);
        np.gridDim = dim3(grid);
        np.blockDim = dim3(block);
        np.sharedMemBytes = 0;
        np.kernelParams = args;
        np.extra = nullptr;
        hipGraphNode_t node;
        e = hipGraphAddKernelNode(&node, graph, prev ? &prev : nullptr, prev ? 1 : 0, &np);
        prev = node;
    }
    hipGraphExec_t exec = nullptr;
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return hip_fail(e, "building the step graph");
    }
    h->graph = graph;
    h->graph_exec = exec;
    return KBC_OK;
}

// ---------------------------------------------------------------------------
// Device scratch of kbc_energy_series_noalloc: a file-scope array in each
// GPU's memory (the runtime places one copy per device when the library's
// code object loads there; it stays until the process ends).  Host code
// reaches it only through the address hipGetSymbolAddress returns for the
// current device: the array's name in host code is not a device address.
//   [0, kScrPartial)                 per-block partial sums of a reduction
//   [kScrPartial, +8)                the sums of u (and spare)
//   [kScrPartial + 8, + max steps)   k after each step, copied out at the end
// Nothing in it has to start at zero: every value is written before it is
// read.  Calls on one GPU share the array.
// ---------------------------------------------------------------------------
constexpr int64_t kNoAllocMaxSteps = KBC_NOALLOC_MAX_STEPS;
constexpr size_t kScrPartial = 3 * 1024;
constexpr size_t kScrSums = 8;
constexpr size_t kScrDoubles = kScrPartial + kScrSums + (size_t)kNoAllocMaxSteps;
constexpr int kMaxDevices = 64;

}  // namespace

static __device__ __align__(256) double scratch[kScrDoubles];

namespace {

std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices];

// Address of this device's copy of `scratch`, looked up once per device with
// that device current (the caller has made it current).
int device_scratch(int dev, double** out)
{
    if (dev < 0 || dev >= kMaxDevices) return fail(KBC_EINVAL, "device ordinal above 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(KBC_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return KBC_OK;
}

// One step as its own launch.
int step_once(kbc_handle h)
{
    StepParams p = step_params(h);
    const int sweep = step_sweep(h, h->cur, h->t, p);
    KBC_HIP(launch_step(h->dtype, h->variant, sweep, h->exact_gamma, p, h->stream));
    if (h->streaming == KBC_PULL) h->cur = 1 - h->cur;
    h->t += 1;
    return KBC_OK;
}

}  // namespace

extern "C" {

void kbc_options_default(kbc_options* opt)
{
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->variant = KBC_S_DTQ;
    opt->streaming = KBC_PULL;
    opt->gamma_mode = KBC_GAMMA_ENTROPIC;
    opt->device = -1;
    opt->gamma_value = 2.0;
    opt->gamma_eps = 0.0;
    opt->stream = nullptr;
}

const char* kbc_last_error(void) { return g_last_error.c_str(); }

int kbc_create(const int64_t shape[3], double nu, int32_t dtype, const kbc_options* opt_in,
               kbc_handle* out)
{
    if (!out) return fail(KBC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!shape) return fail(KBC_EINVAL, "shape is NULL");
    kbc_options opt;
    if (opt_in) opt = *opt_in;
    else kbc_options_default(&opt);
    for (int a = 0; a < 3; ++a)
        if (shape[a] < 1) return fail(KBC_EINVAL, "shape entries must be >= 1");
    const double nn = (double)shape[0] * (double)shape[1] * (double)shape[2];
    if (nn >= 2147483648.0) return fail(KBC_EINVAL, "box has 2^31 nodes or more");
    if (!(nu > 0.0) || !std::isfinite(nu)) return fail(KBC_EINVAL, "nu must be finite and > 0");
    if (dtype != KBC_F64 && dtype != KBC_F32_DEV && dtype != KBC_F16_DEV && dtype != KBC_F32_DEV_X)
        return fail(KBC_EINVAL, "unknown dtype");
    // the step kernels address a node inside a direction plane with a 32-bit
    // byte offset
    if (nn * (double)elem_bytes(dtype) > 4294967296.0)
        return fail(KBC_EINVAL, "a direction plane of this box exceeds 4 GiB (FP64: 2^29 nodes at most)");
    if (opt.variant < KBC_S_D || opt.variant > KBC_S_CDTQ) return fail(KBC_EINVAL, "unknown variant");
    if (opt.streaming != KBC_PULL && opt.streaming != KBC_AA) return fail(KBC_EINVAL, "unknown streaming");
    if (opt.gamma_mode < KBC_GAMMA_ENTROPIC || opt.gamma_mode > KBC_GAMMA_EXACT)
        return fail(KBC_EINVAL, "unknown gamma_mode");
    if (opt.gamma_mode == KBC_GAMMA_FIXED && !std::isfinite(opt.gamma_value))
        return fail(KBC_EINVAL, "gamma_value must be finite");

    kbc_box* h = new (std::nothrow) kbc_box();
    if (!h) return fail(KBC_ENOMEM, "host allocation failed");
    std::memset(h, 0, sizeof(*h));
    for (int a = 0; a < 3; ++a) h->shape[a] = shape[a];
    h->g.nx = (uint32_t)shape[0];
    h->g.ny = (uint32_t)shape[1];
    h->g.nz = (uint32_t)shape[2];
    h->g.nnodes = (uint32_t)(shape[0] * shape[1] * shape[2]);
    h->g.dnx = make_fastdiv(h->g.nx);
    h->g.dny = make_fastdiv(h->g.ny);
    // Pull boxes whose whole lattice lies within 4 GiB (the step kernels'
    // 32-bit offsets) are x-blocked: the 27 populations of 64 (or 32) nodes
    // adjacent in x are contiguous, which measured 5% faster than planes for
    // the FP64 pull step (and the same for AA, which stays in planes).
    // Otherwise planes, spaced by the node count plus a pad that keeps the
    // 27 read and 27 write streams off a common power-of-two stride.
    if (opt.streaming == KBC_PULL && 27.0 * nn * (double)elem_bytes(dtype) < 4294967296.0)
        geom_blocked(h->g);
    else
        geom_planes(h->g, plane_pad_elems(h->g.nnodes, elem_bytes(dtype), opt.streaming));
    h->dtype = dtype;
    h->variant = opt.variant;
    h->streaming = opt.streaming;
    // AA sweeps whose three z-slabs over the 27 planes exceed half of the
    // last-level cache give each XCD one contiguous eighth of the
    // workgroups, the others consecutive pairs (step_block)
    h->xcd_eighths = opt.streaming == KBC_AA &&
                    3.0 * 27.0 * (double)h->g.slab * (double)elem_bytes(dtype) > 128.0 * 1048576.0;
    h->nu = nu;
    // nu = c_s^2 (1/(2 beta) - 1/2), c_s^2 = 1/3
    const double beta = 1.0 / (6.0 * nu + 1.0);
    h->coll.beta = beta;
    h->coll.inv_beta = 1.0 / beta;
    h->coll.c2 = 2.0 - 1.0 / beta;
    h->coll.gamma_eps = opt.gamma_eps > 0.0 ? opt.gamma_eps : (dtype == KBC_F64 ? 1e-28 : 1e-16);
    h->coll.gamma_fixed = opt.gamma_mode == KBC_GAMMA_FIXED ? 1 : 0;
    h->exact_gamma = opt.gamma_mode == KBC_GAMMA_EXACT;
    h->coll.gamma_value = opt.gamma_value;
    for (int i = 0; i < 27; ++i) h->scale[i] = h->inv_scale[i] = 1.0f;
    std::memset(h->scale_exp, 0, sizeof(h->scale_exp));

    int dev = opt.device;
    if (dev < 0) {
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) {
            delete h;
            return hip_fail(e, "hipGetDevice");
        }
    }
    h->device = dev;
    hipError_t e = hipSetDevice(dev);
    if (e != hipSuccess) {
        delete h;
        return hip_fail(e, "hipSetDevice");
    }
    if (opt.stream) {
        h->stream = (hipStream_t)opt.stream;
        h->own_stream = false;
    } else {
        e = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete h;
            return hip_fail(e, "hipStreamCreate");
        }
        h->own_stream = true;
    }
    const size_t bytes = geom_extent(h->g) * elem_bytes(dtype);
    const int nbuf = h->streaming == KBC_PULL ? 2 : 1;
    for (int b = 0; b < nbuf; ++b) {
        e = hipMalloc(&h->buf[b], bytes);
        if (e != hipSuccess) {
            kbc_destroy(h);
            return hip_fail(e, "hipMalloc(populations)");
        }
    }
    *out = h;
    return KBC_OK;
}

int kbc_destroy(kbc_handle h)
{
    if (!h) return KBC_OK;
    (void)hipSetDevice(h->device);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    drop_graph(h);
    for (void* p : {h->buf[0], h->buf[1], (void*)h->d_u, (void*)h->d_rho, (void*)h->d_partial,
                    (void*)h->d_sum, (void*)h->d_flag, (void*)h->d_max, (void*)h->d_pop})
        if (p) (void)hipFree(p);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
    return KBC_OK;
}

static int init_from_device(kbc_handle h, const double* du, const double* drho)
{
    int r = ensure_small(h);
    if (r) return r;
    KBC_HIP(hipMemsetAsync(h->d_flag, 0, sizeof(int), h->stream));
    KBC_HIP(launch_check_init(h->g, du, drho, h->d_flag, h->stream));
    int flag = 0;
    KBC_HIP(hipMemcpyAsync(&flag, h->d_flag, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    KBC_HIP(hipStreamSynchronize(h->stream));
    if (flag)
        return fail(KBC_EUNSTABLE,
                    "initial state has |u_a| >= 1 or rho <= 0 (equilibrium not positive)");
    if (h->dtype == KBC_F16_DEV) {
        KBC_HIP(launch_feq_dev_max(h->g, du, drho, h->d_max, h->stream));
        unsigned mb[27];
        KBC_HIP(hipMemcpyAsync(mb, h->d_max, sizeof(mb), hipMemcpyDeviceToHost, h->stream));
        KBC_HIP(hipStreamSynchronize(h->stream));
        choose_scales(h, mb);
    }
    drop_graph(h);
    h->t = 0;
    h->cur = 0;
    KBC_HIP(launch_init_feq(h->dtype, layout_now(h), state_buf(h), h->g, h->scale, du, drho,
                            h->stream));
    KBC_HIP(hipStreamSynchronize(h->stream));
    h->initialised = true;
    return KBC_OK;
}

int kbc_init_velocity(kbc_handle h, const double* u, const double* rho)
{
    if (int r = check_handle(h)) return r;
    if (!u) return fail(KBC_EINVAL, "u is NULL");
    if (int r = set_device(h)) return r;
    int r = ensure_diag(h, rho != nullptr);
    if (r) return r;
    const size_t N = h->g.nnodes;
    KBC_HIP(hipMemcpyAsync(h->d_u, u, 3 * N * sizeof(double), hipMemcpyHostToDevice, h->stream));
    if (rho) KBC_HIP(hipMemcpyAsync(h->d_rho, rho, N * sizeof(double), hipMemcpyHostToDevice, h->stream));
    return init_from_device(h, h->d_u, rho ? h->d_rho : nullptr);
}

int kbc_init_velocity_device(kbc_handle h, const double* u_dev, const double* rho_dev)
{
    if (int r = check_handle(h)) return r;
    if (!u_dev) return fail(KBC_EINVAL, "u_dev is NULL");
    if (int r = set_device(h)) return r;
    return init_from_device(h, u_dev, rho_dev);
}

int kbc_step(kbc_handle h, int64_t n)
{
    if (int r = check_handle(h)) return r;
    if (n < 0) return fail(KBC_EINVAL, "n must be >= 0");
    if (!h->initialised) return fail(KBC_ESTATE, "box has no state (call kbc_init_velocity)");
    if (n == 0) return KBC_OK;
    if (int r = set_device(h)) return r;
    int64_t left = n;
    if (kStepGraph > 0 && n >= kStepGraph) {
        if (!at_graph_start(h)) {
            if (int r = step_once(h)) return r;
            --left;
        }
        if (left >= kStepGraph && !h->graph_exec)
            if (int r = build_graph(h)) return r;
        for (; left >= kStepGraph; left -= kStepGraph) {
            KBC_HIP(hipGraphLaunch(h->graph_exec, h->stream));
            h->t += kStepGraph;   // and the pull buffers are back where they were
        }
    }
    for (; left > 0; --left)
        if (int r = step_once(h)) return r;
    return KBC_OK;
}

int kbc_moments(kbc_handle h, double* rho, double* u)
{
    if (int r = check_handle(h)) return r;
    if (!h->initialised) return fail(KBC_ESTATE, "box has no state");
    if (int r = set_device(h)) return r;
    const int st = compute_moments(h, rho != nullptr);
    if (st != KBC_OK && st != KBC_EUNSTABLE) return st;
    const size_t N = h->g.nnodes;
    if (rho) KBC_HIP(hipMemcpy(rho, h->d_rho, N * sizeof(double), hipMemcpyDeviceToHost));
    if (u) KBC_HIP(hipMemcpy(u, h->d_u, 3 * N * sizeof(double), hipMemcpyDeviceToHost));
    if (st == KBC_EUNSTABLE) g_last_error = "state is not finite (the run has diverged)";
    return st;
}

static int mean_sums(kbc_handle h)
{
    KBC_HIP(launch_reduce(0, h->g, h->d_u, nullptr, h->d_partial, h->d_sum, h->stream));
    return KBC_OK;
}

int kbc_energy(kbc_handle h, double* k)
{
    if (int r = check_handle(h)) return r;
    if (!k) return fail(KBC_EINVAL, "k is NULL");
    if (!h->initialised) return fail(KBC_ESTATE, "box has no state");
    if (int r = set_device(h)) return r;
    if (int r = compute_moments(h, false)) return r;
    if (int r = mean_sums(h)) return r;
    KBC_HIP(launch_reduce(1, h->g, h->d_u, h->d_sum, h->d_partial, h->d_sum + 3, h->stream));
    double s = 0.0;
    KBC_HIP(hipMemcpyAsync(&s, h->d_sum + 3, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    KBC_HIP(hipStreamSynchronize(h->stream));
    *k = 0.5 * s / (double)h->g.nnodes;
    return KBC_OK;
}

int kbc_energy_series(kbc_handle h, int64_t n, double* k)
{
    if (int r = check_handle(h)) return r;
    if (n < 0) return fail(KBC_EINVAL, "n must be >= 0");
    if (n > 0 && !k) return fail(KBC_EINVAL, "k is NULL");
    if (!h->initialised) return fail(KBC_ESTATE, "box has no state (call kbc_init_velocity)");
    if (n == 0) return KBC_OK;
    if (int r = set_device(h)) return r;
    if (int r = ensure_diag(h, false)) return r;
    double* d_log = nullptr;
    KBC_HIP(hipMalloc(&d_log, (size_t)n * sizeof(double)));
    // the non-finite flag accumulates over the n moment launches
    hipError_t e = hipMemsetAsync(h->d_flag, 0, sizeof(int), h->stream);
    int r = e == hipSuccess ? KBC_OK : hip_fail(e, "hipMemsetAsync");
    for (int64_t j = 0; j < n && r == KBC_OK; ++j) {
        r = kbc_step(h, 1);
        if (r != KBC_OK) break;
        e = launch_moments(h->dtype, layout_now(h), state_buf(h), h->g, h->inv_scale, nullptr,
                           h->d_u, h->d_flag, h->stream);
        if (e == hipSuccess)
            e = launch_reduce(0, h->g, h->d_u, nullptr, h->d_partial, h->d_sum, h->stream);
        if (e == hipSuccess)
            e = launch_reduce(1, h->g, h->d_u, h->d_sum, h->d_partial, h->d_sum + 3, h->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(d_log + j, h->d_sum + 3, sizeof(double), hipMemcpyDeviceToDevice,
                               h->stream);
        if (e != hipSuccess) r = hip_fail(e, "kbc_energy_series");
    }
    int flag = 0;
    if (r == KBC_OK) {
        e = hipMemcpyAsync(k, d_log, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(&flag, h->d_flag, sizeof(int), hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) r = hip_fail(e, "kbc_energy_series");
    }
    (void)hipStreamSynchronize(h->stream);
    (void)hipFree(d_log);
    if (r != KBC_OK) return r;
    const double inv2n = 0.5 / (double)h->g.nnodes;
    for (int64_t j = 0; j < n; ++j) k[j] *= inv2n;
    if (flag) return fail(KBC_EUNSTABLE, "state is not finite (the run has diverged)");
    return KBC_OK;
}

int kbc_energy_series_noalloc(kbc_handle h, int64_t n, double* k)
{
    if (int r = check_handle(h)) return r;
    if (n < 0) return fail(KBC_EINVAL, "n must be >= 0");
    if (n > kNoAllocMaxSteps)
        return fail(KBC_EINVAL, "n exceeds KBC_NOALLOC_MAX_STEPS (65536), the steps the "
                                "static scratch array can log");
    if (n > 0 && !k) return fail(KBC_EINVAL, "k is NULL");
    if (!h->initialised) return fail(KBC_ESTATE, "box has no state (call kbc_init_velocity)");
    if (n == 0) return KBC_OK;
    if (reduce_partials() * 3 > (int)kScrPartial)
        return fail(KBC_EDEVICE, "reduction partials exceed the scratch array");
    if (int r = set_device(h)) return r;
    double* scr = nullptr;
    if (int r = device_scratch(h->device, &scr)) return r;
    double* partial = scr;
    double* sums = scr + kScrPartial;
    double* log = scr + kScrPartial + kScrSums;
    for (int64_t j = 0; j < n; ++j) {
        if (int r = step_once(h)) return r;
        KBC_HIP(launch_energy_direct(h->dtype, layout_now(h), state_buf(h), h->g, h->inv_scale,
                                     partial, sums, log + j, h->stream));
    }
    KBC_HIP(hipMemcpyAsync(k, log, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    KBC_HIP(hipStreamSynchronize(h->stream));
    const double inv2n = 0.5 / (double)h->g.nnodes;
    bool finite = true;
    for (int64_t j = 0; j < n; ++j) {
        k[j] *= inv2n;
        finite = finite && std::isfinite(k[j]);
    }
    if (!finite) return fail(KBC_EUNSTABLE, "state is not finite (the run has diverged)");
    return KBC_OK;
}

int kbc_enstrophy(kbc_handle h, double* omega)
{
    if (int r = check_handle(h)) return r;
    if (!omega) return fail(KBC_EINVAL, "omega is NULL");
    if (!h->initialised) return fail(KBC_ESTATE, "box has no state");
    if (int r = set_device(h)) return r;
    if (int r = compute_moments(h, false)) return r;
    if (int r = mean_sums(h)) return r;
    KBC_HIP(launch_reduce(2, h->g, h->d_u, h->d_sum, h->d_partial, h->d_sum + 3, h->stream));
    double s = 0.0;
    KBC_HIP(hipMemcpyAsync(&s, h->d_sum + 3, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    KBC_HIP(hipStreamSynchronize(h->stream));
    *omega = 0.5 * s / (double)h->g.nnodes;
    return KBC_OK;
}

int kbc_statistics(kbc_handle h, int32_t order, kbc_stats* out)
{
    if (int r = check_handle(h)) return r;
    if (!out) return fail(KBC_EINVAL, "out is NULL");
    if (order != 2 && order != 8) return fail(KBC_EINVAL, "order must be 2 or 8");
    if (!h->initialised) return fail(KBC_ESTATE, "box has no state");
    if (int r = set_device(h)) return r;
    if (int r = compute_moments(h, false)) return r;
    if (int r = mean_sums(h)) return r;
    KBC_HIP(launch_reduce(1, h->g, h->d_u, h->d_sum, h->d_partial, h->d_sum + 3, h->stream));
    KBC_HIP(launch_grad_stats(order, h->g, h->d_u, h->d_partial, h->d_sum + 8, h->stream));
    double s[16];
    KBC_HIP(hipMemcpyAsync(s, h->d_sum, sizeof(s), hipMemcpyDeviceToHost, h->stream));
    KBC_HIP(hipStreamSynchronize(h->stream));
    const double N = (double)h->g.nnodes;
    out->k = 0.5 * s[3] / N;
    out->omega = 0.5 * s[8] / N;
    out->epsilon = 0.5 * h->nu * s[9] / N;
    out->div2 = s[10] / N;
    for (int n = 0; n < 5; ++n) out->dudx_moment[n] = s[11 + n] / N;
    const double m2 = out->dudx_moment[0];
    for (int n = 3; n <= 6; ++n)
        out->skewness[n - 3] = ((n % 2) ? -1.0 : 1.0) * out->dudx_moment[n - 2] / std::pow(m2, 0.5 * n);
    return KBC_OK;
}

int kbc_gamma_statistics(kbc_handle h, double out[4])
{
    if (int r = check_handle(h)) return r;
    if (!out) return fail(KBC_EINVAL, "out is NULL");
    if (!h->initialised) return fail(KBC_ESTATE, "box has no state");
    if (int r = set_device(h)) return r;
    if (int r = ensure_small(h)) return r;
    KBC_HIP(launch_gamma_stats(h->dtype, h->variant, h->exact_gamma, layout_now(h), state_buf(h),
                               h->g, h->coll, h->inv_scale, h->d_partial, h->d_sum + 16,
                               h->stream));
    double s[4];
    KBC_HIP(hipMemcpyAsync(s, h->d_sum + 16, sizeof(s), hipMemcpyDeviceToHost, h->stream));
    KBC_HIP(hipStreamSynchronize(h->stream));
    const double N = (double)h->g.nnodes;
    const double mean = s[0] / N;
    out[0] = mean;
    out[1] = std::sqrt(std::max(0.0, s[1] / N - mean * mean));
    out[2] = s[2];
    out[3] = s[3];
    if (!std::isfinite(mean)) return fail(KBC_EUNSTABLE, "state is not finite (the run has diverged)");
    return KBC_OK;
}

int kbc_correlation(kbc_handle h, int32_t rmax, double* rho11, double* rho22)
{
    if (int r = check_handle(h)) return r;
    if (!rho11 || !rho22) return fail(KBC_EINVAL, "rho11 or rho22 is NULL");
    if (!h->initialised) return fail(KBC_ESTATE, "box has no state");
    if ((int)h->g.nx > corr_max_nx()) return fail(KBC_EINVAL, "nx above the correlation limit (4096)");
    if (rmax < 0 || rmax >= (int)h->g.nx || rmax >= corr_max_lags())
        return fail(KBC_EINVAL, "rmax must be in [0, nx)");
    if (int r = set_device(h)) return r;
    if (int r = compute_moments(h, false)) return r;
    if (int r = mean_sums(h)) return r;
    const size_t L2 = 2 * (size_t)(rmax + 1);
    double* part = nullptr;
    double* dout = nullptr;
    KBC_HIP(hipMalloc(&part, (size_t)corr_blocks(h->g) * L2 * sizeof(double)));
    hipError_t e = hipMalloc(&dout, L2 * sizeof(double));
    std::vector<double> host(L2);
    if (e == hipSuccess) e = launch_corr_x(h->g, h->d_u, h->d_sum, rmax, part, dout, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(host.data(), dout, L2 * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    (void)hipFree(part);
    if (dout) (void)hipFree(dout);
    if (e != hipSuccess) return fail(KBC_EDEVICE, hipGetErrorString(e));
    for (int r = 0; r <= rmax; ++r) {
        rho11[r] = host[2 * r] / host[0];
        rho22[r] = host[2 * r + 1] / host[1];
    }
    return KBC_OK;
}

int kbc_get_populations(kbc_handle h, double* f)
{
    if (int r = check_handle(h)) return r;
    if (!f) return fail(KBC_EINVAL, "f is NULL");
    if (!h->initialised) return fail(KBC_ESTATE, "box has no state");
    if (int r = set_device(h)) return r;
    if (int r = ensure_pop(h)) return r;
    KBC_HIP(launch_gather_pop(h->dtype, layout_now(h), state_buf(h), h->g, h->inv_scale, h->d_pop,
                              h->stream));
    KBC_HIP(hipStreamSynchronize(h->stream));
    KBC_HIP(hipMemcpy(f, h->d_pop, 27ull * h->g.nnodes * sizeof(double), hipMemcpyDeviceToHost));
    return KBC_OK;
}

int kbc_sample_populations(kbc_handle h, const int64_t* nodes, int64_t count, double* f)
{
    if (int r = check_handle(h)) return r;
    if (count < 0 || count > (1 << 24)) return fail(KBC_EINVAL, "count must be in [0, 2^24]");
    if (count == 0) return KBC_OK;
    if (!nodes || !f) return fail(KBC_EINVAL, "nodes or f is NULL");
    if (!h->initialised) return fail(KBC_ESTATE, "box has no state");
    std::vector<uint32_t> idx((size_t)count);
    for (int64_t k = 0; k < count; ++k) {
        if (nodes[k] < 0 || nodes[k] >= (int64_t)h->g.nnodes)
            return fail(KBC_EINVAL, "node index out of range");
        idx[(size_t)k] = (uint32_t)nodes[k];
    }
    if (int r = set_device(h)) return r;
    uint32_t* d_idx = nullptr;
    double* d_out = nullptr;
    hipError_t e = hipMalloc(&d_idx, idx.size() * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc(&d_out, idx.size() * 27 * sizeof(double));
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_idx, idx.data(), idx.size() * sizeof(uint32_t), hipMemcpyHostToDevice,
                           h->stream);
    if (e == hipSuccess)
        e = launch_sample_pop(h->dtype, layout_now(h), state_buf(h), h->g, h->inv_scale, d_idx,
                              (int)count, d_out, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(f, d_out, idx.size() * 27 * sizeof(double), hipMemcpyDeviceToHost,
                           h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (d_idx) (void)hipFree(d_idx);
    if (d_out) (void)hipFree(d_out);
    if (e != hipSuccess) return hip_fail(e, "kbc_sample_populations");
    return KBC_OK;
}

int kbc_set_populations(kbc_handle h, const double* f, int64_t t)
{
    if (int r = check_handle(h)) return r;
    if (!f) return fail(KBC_EINVAL, "f is NULL");
    if (t < 0) return fail(KBC_EINVAL, "t must be >= 0");
    if (int r = set_device(h)) return r;
    if (int r = ensure_pop(h)) return r;
    KBC_HIP(hipStreamSynchronize(h->stream));
    KBC_HIP(hipMemcpy(h->d_pop, f, 27ull * h->g.nnodes * sizeof(double), hipMemcpyHostToDevice));
    if (h->dtype == KBC_F16_DEV && !h->scales_set) {
        KBC_HIP(launch_pop_dev_max(h->g, h->d_pop, h->d_max, h->stream));
        unsigned mb[27];
        KBC_HIP(hipMemcpyAsync(mb, h->d_max, sizeof(mb), hipMemcpyDeviceToHost, h->stream));
        KBC_HIP(hipStreamSynchronize(h->stream));
        choose_scales(h, mb);
    }
    drop_graph(h);
    h->t = t;
    h->cur = 0;
    KBC_HIP(launch_scatter_pop(h->dtype, layout_now(h), state_buf(h), h->g, h->scale, h->d_pop,
                               h->stream));
    KBC_HIP(hipStreamSynchronize(h->stream));
    h->initialised = true;
    return KBC_OK;
}

int kbc_time(kbc_handle h, int64_t* t)
{
    if (int r = check_handle(h)) return r;
    if (!t) return fail(KBC_EINVAL, "t is NULL");
    *t = h->t;
    return KBC_OK;
}

int kbc_sync(kbc_handle h)
{
    if (int r = check_handle(h)) return r;
    if (int r = set_device(h)) return r;
    KBC_HIP(hipStreamSynchronize(h->stream));
    return KBC_OK;
}

int kbc_bytes_per_node_step(kbc_handle h, double* bytes)
{
    if (int r = check_handle(h)) return r;
    if (!bytes) return fail(KBC_EINVAL, "bytes is NULL");
    *bytes = 2.0 * 27.0 * (double)elem_bytes(h->dtype);
    return KBC_OK;
}

int kbc_stream(kbc_handle h, void** stream)
{
    if (int r = check_handle(h)) return r;
    if (!stream) return fail(KBC_EINVAL, "stream is NULL");
    *stream = (void*)h->stream;
    return KBC_OK;
}

int kbc_hbm_copy(void* dst, const void* src, size_t bytes, void* stream)
{
    if (!dst || !src) return fail(KBC_EINVAL, "dst or src is NULL");
    if (bytes % 16) return fail(KBC_EINVAL, "bytes must be a multiple of 16");
    if (dst == src) {
        KBC_HIP(launch_rewrite16(dst, bytes / 16, (hipStream_t)stream));
        return KBC_OK;
    }
    const uintptr_t d = (uintptr_t)dst, s = (uintptr_t)src;
    if (d < s + bytes && s < d + bytes) return fail(KBC_EINVAL, "dst and src overlap");
    KBC_HIP(launch_copy16(dst, src, bytes / 16, (hipStream_t)stream));
    return KBC_OK;
}

}  // extern "C"
