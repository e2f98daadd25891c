// kbc_pool.hip -- batched ensemble ("pool") of independent periodic boxes
// for continuous batching (declared in include/kbc.h).
//
// A pool owns one HBM arena sized by the caller's budget.  Each admitted box
// gets a contiguous region of the arena holding its populations in the AA
// in-place layout (one lattice).  A batch of g steps advances every
// unfinished box by up to g steps.  The boxes of a batch are split into
// launch groups: boxes at the same AA parity whose populations together fit
// the GPU's last-level cache (256 MB on MI355X), largest first.  A group
// takes all g of its steps, one launch of the pool kernel per step (a
// persistent grid-stride loop over the tiles of the group's boxes), before
// the next group starts, so from its second step on a group works out of
// the cache instead of HBM.  The launches are captured once in a hipGraph
// and replayed; the box table and group table the kernels read live at
// fixed device addresses and are uploaded before each batch, so admissions
// and releases never invalidate a graph.  Boxes differ in size, viscosity
// and step count.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <new>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "kbc.h"
#include "kbc_internal.h"

using namespace kbc;

namespace {

int pfail(int code, const std::string& msg)
{
    set_last_error(msg.c_str());
    return code;
}

int phip(hipError_t e, const char* where)
{
    if (e == hipErrorOutOfMemory) return pfail(KBC_ENOMEM, std::string(where) + ": out of device memory");
    return pfail(KBC_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

#define PHIP(call)                                          \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return phip(e_, #call);       \
    } while (0)

size_t elem_bytes_of(int dtype) { return dtype == KBC_F64 ? 8 : (dtype == KBC_F16_DEV ? 2 : 4); }

// First-fit allocator over [0, size) in units of kGrain bytes; free blocks
// are kept by offset and coalesced on release.
class Arena {
public:
    static constexpr size_t kGrain = 65536;
    void reset(size_t size)
    {
        free_.clear();
        size_ = size / kGrain * kGrain;
        if (size_) free_[0] = size_;
        used_ = 0;
    }
    bool alloc(size_t bytes, size_t* off)
    {
        const size_t need = (bytes + kGrain - 1) / kGrain * kGrain;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= need) {
                *off = it->first;
                const size_t rest = it->second - need;
                const size_t start = it->first + need;
                free_.erase(it);
                if (rest) free_[start] = rest;
                used_ += need;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        const size_t need = (bytes + kGrain - 1) / kGrain * kGrain;
        used_ -= need;
        auto it = free_.emplace(off, need).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }
    size_t size() const { return size_; }

private:
    std::map<size_t, size_t> free_;
    size_t size_ = 0, used_ = 0;
};

struct Event {
    hipEvent_t e = nullptr;
    ~Event()
    {
        if (e) (void)hipEventDestroy(e);
    }
    bool done() const { return hipEventQuery(e) == hipSuccess; }
};

struct Slot {
    bool used = false;
    Geom g{};
    Coll c{};
    size_t off = 0, bytes = 0;
    int64_t t = 0;          // steps enqueued
    int64_t t_prev = 0;     // steps enqueued before the last batch
    int64_t target = 0;     // steps requested
    std::shared_ptr<Event> last;
    float scale[27], inv_scale[27];
    int8_t scale_exp[28];
};

struct LaunchCfg {
    int block, grid, sub;   // threads per block, blocks (0: one per tile), sub-tiles per tile
    bool one = false;       // a block for every tile and sub = 1: the single-tile kernel
};

// Launch groups: target footprint (populations of the group's boxes, a
// little below the 256 MB last-level cache) and the most groups per parity.
// The ensemble pool step measured 25.7-27.5 GLUPS (FP32) on 180-220 MiB of
// boxes against 22.9-23.5 on 360 MiB and more.
#ifndef KBC_POOL_GROUP_MIB
#define KBC_POOL_GROUP_MIB 216
#endif
constexpr size_t kGroupBytes = (size_t)KBC_POOL_GROUP_MIB << 20;
constexpr int kMaxGroupsPerParity = 80;

// Blocks of a launch: the persistent grid, or one block per tile rounded up
// to a multiple of 2048 (few distinct graphs; spare blocks exit at once).
int launch_grid(const LaunchCfg& cfg, uint32_t tiles)
{
    if (cfg.grid > 0) return cfg.grid;
    const uint32_t t = std::max<uint32_t>(tiles, 1);
    return (int)((t + 2047) / 2048 * 2048);
}

}  // namespace

struct kbc_pool {
    int dtype = 0, variant = KBC_S_DTQ, device = 0;
    Coll defaults{};
    hipStream_t stream = nullptr, admit_stream = nullptr, diag_stream = nullptr;
    bool own_stream = false;
    char* arena_base = nullptr;
    Arena arena;
    std::vector<Slot> slots;
    // box table (one entry per box of a batch), its tile starts and the
    // group table; the host side is double-buffered (mirror m)
    PoolBox* d_boxes = nullptr;
    uint32_t* d_tstart = nullptr;
    PoolMeta* d_meta = nullptr;
    PoolBox* h_boxes[2] = {nullptr, nullptr};
    uint32_t* h_tstart[2] = {nullptr, nullptr};
    PoolMeta* h_meta[2] = {nullptr, nullptr};
    hipEvent_t mirror_ev[2] = {nullptr, nullptr};
    bool mirror_used[2] = {false, false};
    int mirror = 0;
    // graphs keyed by (steps, block, grid, single-tile kernel, groups at
    // parity 0, at parity 1)
    using GraphKey = std::tuple<int64_t, int, int, bool, int, int>;
    std::map<GraphKey, hipGraphExec_t> graphs;
    std::vector<GraphKey> graph_order;
    LaunchCfg cfg{256, 0, 1};          // the configuration of the latest batch
    bool fixed = false;                // set by kbc_pool_set_launch
    std::map<int, LaunchCfg> tuned;    // box-size bucket -> chosen configuration
    bool tuning = false;               // a tuning round is in progress
    int tune_bucket = -1;              // the bucket it measures
    std::vector<LaunchCfg> cands;
    std::vector<double> cand_cost;
    size_t cand_next = 0;
    hipEvent_t tev0 = nullptr, tev1 = nullptr;
    bool timing_pending = false;
    int timing_cand = -1;
    double timing_node_steps = 0;
    std::string tune_cache;
    int cus = 256;
    // staging and diagnostics scratch (grown on demand)
    double* d_stage = nullptr;
    size_t stage_cap = 0;
    double* d_u = nullptr;
    size_t u_cap = 0;
    double* d_rho = nullptr;
    double* d_partial = nullptr;
    double* d_sum = nullptr;
    int* d_flag = nullptr;
    unsigned* d_max = nullptr;
};

namespace {

int ensure_stage(kbc_pool* p, size_t nnodes)
{
    if (p->stage_cap < nnodes) {
        if (p->d_stage) PHIP(hipFree(p->d_stage));
        p->d_stage = nullptr;
        PHIP(hipMalloc(&p->d_stage, 3 * nnodes * sizeof(double)));
        p->stage_cap = nnodes;
    }
    return KBC_OK;
}

int ensure_diag(kbc_pool* p, size_t nnodes)
{
    if (p->u_cap < nnodes) {
        if (p->d_u) PHIP(hipFree(p->d_u));
        if (p->d_rho) PHIP(hipFree(p->d_rho));
        p->d_u = nullptr;
        p->d_rho = nullptr;
        PHIP(hipMalloc(&p->d_u, 3 * nnodes * sizeof(double)));
        PHIP(hipMalloc(&p->d_rho, nnodes * sizeof(double)));
        p->u_cap = nnodes;
    }
    return KBC_OK;
}

// Tuned configurations are kept per workload class: the bucket of a batch is
// floor(log2(mean nodes per box)), since the best tile and grid shape differ
// between many small boxes and a few large ones.
std::string cache_prefix(const kbc_pool* p)
{
    std::ostringstream os;
    os << "gfx950 dtype=" << p->dtype << " variant=" << p->variant << " bucket=";
    return os.str();
}

void load_tune_cache(kbc_pool* p)
{
    if (p->tune_cache.empty()) return;
    std::ifstream in(p->tune_cache);
    std::string line;
    const std::string pre = cache_prefix(p);
    while (std::getline(in, line)) {
        const size_t bar = line.find('|');
        if (bar == std::string::npos || line.compare(0, pre.size(), pre) != 0) continue;
        std::istringstream key(line.substr(pre.size(), bar - pre.size()));
        std::istringstream rest(line.substr(bar + 1));
        int bucket = -1, block = 0, grid = 0, sub = 0;
        if (key >> bucket && rest >> block >> grid >> sub && bucket >= 0 && bucket < 40 &&
            block >= 64 && block <= kPoolMaxBlock && block % 64 == 0 && grid >= 0 && sub >= 1 &&
            sub <= 64)
            p->tuned[bucket] = LaunchCfg{block, grid, sub};
    }
}

void save_tune_cache(kbc_pool* p)
{
    if (p->tune_cache.empty()) return;
    std::vector<std::string> keep;
    const std::string pre = cache_prefix(p);
    {
        std::ifstream in(p->tune_cache);
        std::string line;
        while (std::getline(in, line))
            if (!line.empty() && line.compare(0, pre.size(), pre) != 0) keep.push_back(line);
    }
    std::ofstream out(p->tune_cache, std::ios::trunc);
    for (auto& l : keep) out << l << "\n";
    for (auto& kv : p->tuned)
        out << pre << kv.first << "|" << kv.second.block << " " << kv.second.grid << " "
            << kv.second.sub << "\n";
}

// Collect a finished timing measurement of the online tuner, if any.
void tuner_collect(kbc_pool* p, bool wait)
{
    if (!p->timing_pending) return;
    if (!wait && hipEventQuery(p->tev1) != hipSuccess) return;
    (void)hipEventSynchronize(p->tev1);
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, p->tev0, p->tev1) == hipSuccess && p->timing_node_steps > 0) {
        const double cost = ms / p->timing_node_steps;
        double& slot = p->cand_cost[p->timing_cand];
        slot = std::min(slot, cost);
    }
    p->timing_pending = false;
    // every candidate is timed twice (the first batch of a new graph also
    // uploads it); the better of the two counts
    if (p->cand_next >= 2 * p->cands.size()) {
        size_t best = 0;
        for (size_t i = 1; i < p->cands.size(); ++i)
            if (p->cand_cost[i] < p->cand_cost[best]) best = i;
        p->tuned[p->tune_bucket] = p->cands[best];
        p->tuning = false;
        save_tune_cache(p);
    }
}

void destroy_graphs(kbc_pool* p)
{
    for (auto& kv : p->graphs) (void)hipGraphExecDestroy(kv.second);
    p->graphs.clear();
    p->graph_order.clear();
}

// n0 launch groups at parity 0 (table entries 0 .. n0-1), then n1 at parity
// 1: each group takes its `steps` steps before the next group starts.
int get_graph(kbc_pool* p, int64_t steps, LaunchCfg cfg, int n0, int n1, hipGraphExec_t* out)
{
    // the sub-tile count lives in the uploaded table, not in the graph; the
    // graph depends on it only through the choice of the single-tile kernel
    const auto key = std::make_tuple(steps, cfg.block, cfg.grid, cfg.one, n0, n1);
    auto it = p->graphs.find(key);
    if (it != p->graphs.end()) {
        *out = it->second;
        return KBC_OK;
    }
    if (p->graphs.size() >= 64) {
        const auto old = p->graph_order.front();
        p->graph_order.erase(p->graph_order.begin());
        (void)hipGraphExecDestroy(p->graphs[old]);
        p->graphs.erase(old);
    }
    hipGraph_t graph = nullptr;
    PHIP(hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal));
    hipError_t err = hipSuccess;
    for (int grp = 0; grp < n0 + n1 && err == hipSuccess; ++grp) {
        const int parity = grp < n0 ? 0 : 1;
        for (int64_t k = 0; k < steps && err == hipSuccess; ++k) {
            // a box at parity q takes the even sweep at steps k with k + q even
            const int sweep = ((parity + k) & 1) ? SW_AA_ODD : SW_AA_EVEN;
            err = launch_pool_step(p->dtype, p->variant, sweep, p->d_boxes, p->d_tstart,
                                   p->d_meta + grp, (int)k, cfg.block, cfg.grid, cfg.one,
                                   p->stream);
        }
    }
    const hipError_t e2 = hipStreamEndCapture(p->stream, &graph);
    if (err != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return phip(err, "pool step capture");
    }
    if (e2 != hipSuccess) return phip(e2, "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    const hipError_t e3 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e3 != hipSuccess) return phip(e3, "hipGraphInstantiate");
    p->graphs[key] = exec;
    p->graph_order.push_back(key);
    *out = exec;
    return KBC_OK;
}

int check_pool(kbc_pool_handle p)
{
    if (!p) return pfail(KBC_EINVAL, "null pool");
    return KBC_OK;
}

int check_slot(kbc_pool_handle p, int32_t slot)
{
    if (int r = check_pool(p)) return r;
    if (slot < 0 || slot >= (int32_t)p->slots.size() || !p->slots[slot].used)
        return pfail(KBC_EINVAL, "no box in this slot");
    return KBC_OK;
}

}  // namespace

extern "C" {

int kbc_pool_create(size_t hbm_budget_bytes, int32_t dtype, const kbc_options* opt_in,
                    int32_t max_slots, const char* tune_cache, kbc_pool_handle* out)
{
    if (!out) return pfail(KBC_EINVAL, "out is NULL");
    *out = nullptr;
    kbc_options opt;
    if (opt_in) opt = *opt_in;
    else kbc_options_default(&opt);
    if (dtype != KBC_F64 && dtype != KBC_F32_DEV && dtype != KBC_F16_DEV && dtype != KBC_F32_DEV_X)
        return pfail(KBC_EINVAL, "unknown dtype");
    if (opt.variant < KBC_S_D || opt.variant > KBC_S_CDTQ) return pfail(KBC_EINVAL, "unknown variant");
    if (max_slots < 1 || max_slots > 65536) return pfail(KBC_EINVAL, "max_slots must be in [1, 65536]");
    if (hbm_budget_bytes < Arena::kGrain) return pfail(KBC_EINVAL, "budget below 64 KiB");
    if (opt.gamma_mode == KBC_GAMMA_EXACT)
        return pfail(KBC_EINVAL, "the exact stabilizer is available for single boxes only");
    if (opt.gamma_mode < KBC_GAMMA_ENTROPIC || opt.gamma_mode > KBC_GAMMA_FIXED)
        return pfail(KBC_EINVAL, "unknown gamma_mode");
    if (opt.gamma_mode == KBC_GAMMA_FIXED && !std::isfinite(opt.gamma_value))
        return pfail(KBC_EINVAL, "gamma_value must be finite");

    std::unique_ptr<kbc_pool> p(new (std::nothrow) kbc_pool());
    if (!p) return pfail(KBC_ENOMEM, "host allocation failed");
    p->dtype = dtype;
    p->variant = opt.variant;
    p->defaults.gamma_fixed = opt.gamma_mode == KBC_GAMMA_FIXED ? 1 : 0;
    p->defaults.gamma_value = opt.gamma_value;
    p->defaults.gamma_eps = opt.gamma_eps > 0.0 ? opt.gamma_eps : (dtype == KBC_F64 ? 1e-28 : 1e-16);
    int dev = opt.device;
    if (dev < 0) PHIP(hipGetDevice(&dev));
    p->device = dev;
    PHIP(hipSetDevice(dev));
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
        p->cus = prop.multiProcessorCount;
    p->cfg = LaunchCfg{256, 0, 1};
    if (opt.stream) {
        p->stream = (hipStream_t)opt.stream;
    } else {
        PHIP(hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking));
        p->own_stream = true;
    }
    PHIP(hipStreamCreateWithFlags(&p->admit_stream, hipStreamNonBlocking));
    PHIP(hipStreamCreateWithFlags(&p->diag_stream, hipStreamNonBlocking));
    const hipError_t ea = hipMalloc(&p->arena_base, hbm_budget_bytes);
    if (ea != hipSuccess) {
        kbc_pool_destroy(p.release());
        return phip(ea, "hipMalloc(arena)");
    }
    p->arena.reset(hbm_budget_bytes);
    p->slots.resize((size_t)max_slots);
    {
        const size_t ngroups = 2 * kMaxGroupsPerParity;
        hipError_t e = hipMalloc(&p->d_boxes, (size_t)max_slots * sizeof(PoolBox));
        if (e == hipSuccess) e = hipMalloc(&p->d_tstart, (size_t)max_slots * sizeof(uint32_t));
        if (e == hipSuccess) e = hipMalloc(&p->d_meta, ngroups * sizeof(PoolMeta));
        for (int m = 0; m < 2 && e == hipSuccess; ++m) {
            e = hipHostMalloc((void**)&p->h_boxes[m], (size_t)max_slots * sizeof(PoolBox));
            if (e == hipSuccess)
                e = hipHostMalloc((void**)&p->h_tstart[m], (size_t)max_slots * sizeof(uint32_t));
            if (e == hipSuccess) e = hipHostMalloc((void**)&p->h_meta[m], ngroups * sizeof(PoolMeta));
        }
        if (e != hipSuccess) {
            kbc_pool_destroy(p.release());
            return phip(e, "pool tables");
        }
    }
    hipError_t e = hipSuccess;
    for (int m = 0; m < 2 && e == hipSuccess; ++m)
        e = hipEventCreateWithFlags(&p->mirror_ev[m], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreate(&p->tev0);
    if (e == hipSuccess) e = hipEventCreate(&p->tev1);
    if (e == hipSuccess) e = hipMalloc(&p->d_partial, 3 * (size_t)reduce_partials() * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&p->d_sum, 8 * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&p->d_flag, sizeof(int));
    if (e == hipSuccess) e = hipMalloc(&p->d_max, 27 * sizeof(unsigned));
    if (e != hipSuccess) {
        kbc_pool_destroy(p.release());
        return phip(e, "pool scratch");
    }
    // tuner candidates: block sizes x (one block per tile | persistent grid)
    // x sub-tiles
    for (int block : {256, 512})
        for (int mult : {0, 16})
            for (int sub : {1, 2, 4}) p->cands.push_back(LaunchCfg{block, mult * p->cus, sub});
    p->cand_cost.assign(p->cands.size(), 1e300);
    p->tuning = false;   // rounds start per box-size bucket, on first use
    if (tune_cache) p->tune_cache = tune_cache;
    load_tune_cache(p.get());
    *out = p.release();
    return KBC_OK;
}

int kbc_pool_destroy(kbc_pool_handle p)
{
    if (!p) return KBC_OK;
    (void)hipSetDevice(p->device);
    if (p->stream) (void)hipStreamSynchronize(p->stream);
    if (p->admit_stream) (void)hipStreamSynchronize(p->admit_stream);
    if (p->diag_stream) (void)hipStreamSynchronize(p->diag_stream);
    destroy_graphs(p);
    for (auto& s : p->slots) s.last.reset();
    for (void* q : {(void*)p->d_boxes, (void*)p->d_tstart, (void*)p->d_meta})
        if (q) (void)hipFree(q);
    for (int m = 0; m < 2; ++m)
        for (void* q : {(void*)p->h_boxes[m], (void*)p->h_tstart[m], (void*)p->h_meta[m]})
            if (q) (void)hipHostFree(q);
    for (int m = 0; m < 2; ++m)
        if (p->mirror_ev[m]) (void)hipEventDestroy(p->mirror_ev[m]);
    if (p->tev0) (void)hipEventDestroy(p->tev0);
    if (p->tev1) (void)hipEventDestroy(p->tev1);
    for (void* q : {(void*)p->arena_base, (void*)p->d_stage, (void*)p->d_u, (void*)p->d_rho,
                    (void*)p->d_partial, (void*)p->d_sum, (void*)p->d_flag, (void*)p->d_max})
        if (q) (void)hipFree(q);
    if (p->admit_stream) (void)hipStreamDestroy(p->admit_stream);
    if (p->diag_stream) (void)hipStreamDestroy(p->diag_stream);
    if (p->own_stream && p->stream) (void)hipStreamDestroy(p->stream);
    delete p;
    return KBC_OK;
}

int kbc_pool_admit(kbc_pool_handle p, const int64_t shape[3], double nu, const double* u,
                   int64_t steps, int32_t* slot_out)
{
    if (int r = check_pool(p)) return r;
    if (!shape || !u || !slot_out) return pfail(KBC_EINVAL, "shape, u or slot is NULL");
    *slot_out = -1;
    for (int a = 0; a < 3; ++a)
        if (shape[a] < 1) return pfail(KBC_EINVAL, "shape entries must be >= 1");
    const double nn = (double)shape[0] * (double)shape[1] * (double)shape[2];
    if (nn >= 2147483648.0) return pfail(KBC_EINVAL, "box has 2^31 nodes or more");
    if (!(nu > 0.0) || !std::isfinite(nu)) return pfail(KBC_EINVAL, "nu must be finite and > 0");
    if (steps < 0) return pfail(KBC_EINVAL, "steps must be >= 0");
    // 32-bit byte offsets inside a direction plane, as in the single-box path
    if (nn * (double)elem_bytes_of(p->dtype) > 4294967296.0)
        return pfail(KBC_EINVAL, "a direction plane of this box exceeds 4 GiB");
    int32_t slot = -1;
    for (size_t i = 0; i < p->slots.size(); ++i)
        if (!p->slots[i].used) {
            slot = (int32_t)i;
            break;
        }
    if (slot < 0) return pfail(KBC_ECAPACITY, "all pool slots are in use");
    const uint64_t nnodes = (uint64_t)(shape[0] * shape[1] * shape[2]);
    const size_t bytes = 27ull * nnodes * elem_bytes_of(p->dtype);
    size_t off = 0;
    if (!p->arena.alloc(bytes, &off)) return pfail(KBC_ECAPACITY, "HBM budget exhausted");
    PHIP(hipSetDevice(p->device));
    Slot s;
    s.g.nx = (uint32_t)shape[0];
    s.g.ny = (uint32_t)shape[1];
    s.g.nz = (uint32_t)shape[2];
    s.g.nnodes = (uint32_t)nnodes;
    s.g.dnx = make_fastdiv(s.g.nx);
    s.g.dny = make_fastdiv(s.g.ny);
    geom_planes(s.g, 0);   // the pool's sweeps are AA
    s.c = p->defaults;
    const double beta = 1.0 / (6.0 * nu + 1.0);  // nu = (1/3)(1/(2 beta) - 1/2)
    s.c.beta = beta;
    s.c.inv_beta = 1.0 / beta;
    s.c.c2 = 2.0 - 1.0 / beta;
    s.off = off;
    s.bytes = bytes;
    s.target = steps;
    for (int i = 0; i < 27; ++i) s.scale[i] = s.inv_scale[i] = 1.0f;
    std::memset(s.scale_exp, 0, sizeof(s.scale_exp));
    auto undo = [&](int code) {
        p->arena.release(off, bytes);
        return code;
    };
    if (int r = ensure_stage(p, nnodes)) return undo(r);
    void* buf = p->arena_base + off;
    hipError_t e = hipMemcpyAsync(p->d_stage, u, 3 * nnodes * sizeof(double), hipMemcpyHostToDevice,
                                  p->admit_stream);
    if (e == hipSuccess) e = hipMemsetAsync(p->d_flag, 0, sizeof(int), p->admit_stream);
    if (e == hipSuccess) e = launch_check_init(s.g, p->d_stage, nullptr, p->d_flag, p->admit_stream);
    int flag = 0;
    if (e == hipSuccess)
        e = hipMemcpyAsync(&flag, p->d_flag, sizeof(int), hipMemcpyDeviceToHost, p->admit_stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->admit_stream);
    if (e != hipSuccess) return undo(phip(e, "kbc_pool_admit"));
    if (flag) return undo(pfail(KBC_EUNSTABLE, "initial state has |u_a| >= 1 (equilibrium not positive)"));
    if (p->dtype == KBC_F16_DEV) {
        unsigned mb[27];
        e = launch_feq_dev_max(s.g, p->d_stage, nullptr, p->d_max, p->admit_stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(mb, p->d_max, sizeof(mb), hipMemcpyDeviceToHost, p->admit_stream);
        if (e == hipSuccess) e = hipStreamSynchronize(p->admit_stream);
        if (e != hipSuccess) return undo(phip(e, "kbc_pool_admit scales"));
        for (int i = 0; i < 27; ++i) {
            float m0, m1;
            std::memcpy(&m0, &mb[i], sizeof(float));
            std::memcpy(&m1, &mb[26 - i], sizeof(float));
            double m = std::max<double>(m0, m1);
            m = std::max(m, 1e-4 * weight(i));
            // within the int8 range, and defined for a non-finite maximum
            const int ex = (int)std::min(126.0, std::max(-126.0, std::floor(std::log2(4096.0 / m))));
            s.scale[i] = std::ldexp(1.0f, ex);
            s.inv_scale[i] = std::ldexp(1.0f, -ex);
            s.scale_exp[i] = (int8_t)ex;
        }
    }
    e = launch_init_feq(p->dtype, LY_AA_EVEN, buf, s.g, s.scale, p->d_stage, nullptr, p->admit_stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->admit_stream);
    if (e != hipSuccess) return undo(phip(e, "kbc_pool_admit init"));
    s.used = true;
    p->slots[slot] = s;
    *slot_out = slot;
    return KBC_OK;
}

static int pool_advance(kbc_pool_handle p, int64_t g, const int32_t* only, int32_t n_only)
{
    if (int r = check_pool(p)) return r;
    if (g < 1 || g > 4096) return pfail(KBC_EINVAL, "g must be in [1, 4096]");
    std::vector<char> pick;
    if (only) {
        pick.assign(p->slots.size(), 0);
        for (int32_t i = 0; i < n_only; ++i) {
            if (only[i] < 0 || only[i] >= (int32_t)p->slots.size() || !p->slots[only[i]].used)
                return pfail(KBC_EINVAL, "slot list names an empty slot");
            pick[only[i]] = 1;
        }
    }
    PHIP(hipSetDevice(p->device));
    // while tuning, each batch times one candidate: wait for the previous one
    tuner_collect(p, p->tuning);
    // the batch's workload class
    double sel_nodes = 0.0;
    int sel_boxes = 0;
    for (size_t si = 0; si < p->slots.size(); ++si) {
        const Slot& s = p->slots[si];
        if (!s.used || s.t >= s.target || (only && !pick[si])) continue;
        sel_nodes += (double)s.g.nnodes;
        ++sel_boxes;
    }
    const int bucket =
        sel_boxes ? std::max(0, (int)std::floor(std::log2(sel_nodes / sel_boxes))) : 0;
    LaunchCfg cfg{256, 0, 1};
    int cand = -1;
    if (p->fixed) {
        cfg = p->cfg;
    } else if (p->tuned.count(bucket)) {
        cfg = p->tuned[bucket];
    } else if (sel_boxes) {
        if (!p->tuning) {
            p->tuning = true;
            p->tune_bucket = bucket;
            p->cand_next = 0;
            p->cand_cost.assign(p->cands.size(), 1e300);
        }
        if (p->tune_bucket == bucket && !p->timing_pending &&
            p->cand_next < 2 * p->cands.size()) {
            cand = (int)(p->cand_next++ % p->cands.size());
            cfg = p->cands[cand];
        }
    }
    p->cfg = cfg;
    const uint32_t tile_nodes = (uint32_t)(cfg.block * cfg.sub);
    // launch groups and their box tables for this batch
    const int m = p->mirror;
    if (p->mirror_used[m]) PHIP(hipEventSynchronize(p->mirror_ev[m]));
    struct Pick {
        size_t si;
        int64_t steps;
    };
    std::vector<Pick> by_parity[2];
    size_t parity_bytes[2] = {0, 0};
    int64_t batch = 0;
    double node_steps = 0.0;
    std::vector<int64_t> adv(p->slots.size(), 0);
    for (size_t si = 0; si < p->slots.size(); ++si) {
        const Slot& s = p->slots[si];
        if (!s.used || s.t >= s.target || (only && !pick[si])) continue;
        const int64_t steps = std::min<int64_t>(g, s.target - s.t);
        by_parity[s.t & 1].push_back(Pick{si, steps});
        parity_bytes[s.t & 1] += s.bytes;
        batch = std::max(batch, steps);
        node_steps += (double)s.g.nnodes * (double)steps;
        adv[si] = steps;
    }
    if (batch == 0) return KBC_OK;
    // largest boxes first, then next fit: a group is closed when the next box
    // would take it past the target footprint (a box above the target forms
    // a group of its own).  With the target raised to 1/32 of the parity's
    // total, next fit makes at most 2 x 32 + 1 groups.
    int ngroups[2] = {0, 0};
    uint32_t nbox = 0, max_tiles = 0;
    for (int par = 0; par < 2; ++par) {
        auto& v = by_parity[par];
        std::stable_sort(v.begin(), v.end(), [&](const Pick& x, const Pick& y) {
            return p->slots[x.si].bytes > p->slots[y.si].bytes;
        });
        const size_t cap = std::max(kGroupBytes, parity_bytes[par] / 32 + 1);
        size_t fill = 0;
        PoolMeta* mt = nullptr;
        for (const Pick& pk : v) {
            const Slot& s = p->slots[pk.si];
            if (!mt || fill + s.bytes > cap) {
                // the parity-1 groups follow the parity-0 groups in the table
                const int gi = (par ? ngroups[0] : 0) + ngroups[par];
                if (ngroups[par] >= kMaxGroupsPerParity) return pfail(KBC_EDEVICE, "pool group table full");
                mt = &p->h_meta[m][gi];
                *mt = PoolMeta{nbox, 0, 0, (uint32_t)cfg.block, (uint32_t)cfg.sub};
                ++ngroups[par];
                fill = 0;
            }
            fill += s.bytes;
            PoolBox& bx = p->h_boxes[m][nbox];
            p->h_tstart[m][nbox] = mt->n_tiles;
            bx.buf = p->arena_base + s.off;
            bx.g = s.g;
            bx.c = s.c;
            bx.tile0 = mt->n_tiles;
            bx.ntiles = (s.g.nnodes + tile_nodes - 1) / tile_nodes;
            bx.parity0 = (int32_t)par;
            bx.steps = (int32_t)pk.steps;
            static_assert(sizeof(bx.scale_exp) == sizeof(s.scale_exp), "exponent layout");
            std::memcpy(bx.scale_exp, s.scale_exp, sizeof(bx.scale_exp));
            mt->n_tiles += bx.ntiles;
            ++mt->n_active;
            max_tiles = std::max(max_tiles, mt->n_tiles);
            ++nbox;
        }
    }
    const int nmeta = ngroups[0] + ngroups[1];
    PHIP(hipMemcpyAsync(p->d_boxes, p->h_boxes[m], nbox * sizeof(PoolBox), hipMemcpyHostToDevice,
                        p->stream));
    PHIP(hipMemcpyAsync(p->d_tstart, p->h_tstart[m], nbox * sizeof(uint32_t), hipMemcpyHostToDevice,
                        p->stream));
    PHIP(hipMemcpyAsync(p->d_meta, p->h_meta[m], nmeta * sizeof(PoolMeta), hipMemcpyHostToDevice,
                        p->stream));
    PHIP(hipEventRecord(p->mirror_ev[m], p->stream));
    p->mirror_used[m] = true;
    p->mirror = 1 - m;

    hipGraphExec_t exec = nullptr;
    LaunchCfg gcfg = cfg;
    gcfg.grid = launch_grid(cfg, max_tiles);
    // one block per tile (the grid covers the largest group) and no sub-tiles
    gcfg.one = cfg.grid == 0 && cfg.sub == 1;
    if (int r = get_graph(p, batch, gcfg, ngroups[0], ngroups[1], &exec)) return r;
    if (cand >= 0) PHIP(hipEventRecord(p->tev0, p->stream));
    PHIP(hipGraphLaunch(exec, p->stream));
    if (cand >= 0) {
        PHIP(hipEventRecord(p->tev1, p->stream));
        p->timing_pending = true;
        p->timing_cand = cand;
        p->timing_node_steps = node_steps;
    }
    auto ev = std::make_shared<Event>();
    PHIP(hipEventCreateWithFlags(&ev->e, hipEventDisableTiming));
    PHIP(hipEventRecord(ev->e, p->stream));
    for (size_t si = 0; si < p->slots.size(); ++si) {
        if (!adv[si]) continue;
        Slot& s = p->slots[si];
        s.t_prev = s.t;
        s.t += adv[si];
        s.last = ev;
    }
    return KBC_OK;
}

int kbc_pool_advance(kbc_pool_handle p, int64_t g) { return pool_advance(p, g, nullptr, 0); }

int kbc_pool_advance_slots(kbc_pool_handle p, int64_t g, const int32_t* slots, int32_t count)
{
    if (count < 0 || (count > 0 && !slots)) return pfail(KBC_EINVAL, "bad slot list");
    if (count == 0) return check_pool(p);
    return pool_advance(p, g, slots, count);
}

int kbc_pool_poll(kbc_pool_handle p, int32_t slot, int64_t* remaining)
{
    if (int r = check_slot(p, slot)) return r;
    if (!remaining) return pfail(KBC_EINVAL, "remaining is NULL");
    const Slot& s = p->slots[slot];
    const int64_t completed = (!s.last || s.last->done()) ? s.t : s.t_prev;
    *remaining = s.target - completed;
    return KBC_OK;
}

int kbc_pool_result(kbc_pool_handle p, int32_t slot, double* k, double* omega, double* rho, double* u)
{
    if (int r = check_slot(p, slot)) return r;
    Slot& s = p->slots[slot];
    if (s.t < s.target) return pfail(KBC_ESTATE, "the box has steps left to run");
    PHIP(hipSetDevice(p->device));
    if (int r = ensure_diag(p, s.g.nnodes)) return r;
    if (s.last) PHIP(hipStreamWaitEvent(p->diag_stream, s.last->e, 0));
    const void* buf = p->arena_base + s.off;
    const int layout = (s.t % 2 == 0) ? LY_AA_EVEN : LY_AA_ODD;
    const int storage = p->dtype == KBC_F32_DEV_X ? KBC_F32_DEV : p->dtype;
    PHIP(hipMemsetAsync(p->d_flag, 0, sizeof(int), p->diag_stream));
    PHIP(launch_moments(storage, layout, buf, s.g, s.inv_scale, p->d_rho, p->d_u, p->d_flag,
                        p->diag_stream));
    PHIP(launch_reduce(0, s.g, p->d_u, nullptr, p->d_partial, p->d_sum, p->diag_stream));
    PHIP(launch_reduce(1, s.g, p->d_u, p->d_sum, p->d_partial, p->d_sum + 3, p->diag_stream));
    PHIP(launch_reduce(2, s.g, p->d_u, p->d_sum, p->d_partial, p->d_sum + 6, p->diag_stream));
    double sums[8];
    int flag = 0;
    PHIP(hipMemcpyAsync(sums, p->d_sum, sizeof(sums), hipMemcpyDeviceToHost, p->diag_stream));
    PHIP(hipMemcpyAsync(&flag, p->d_flag, sizeof(int), hipMemcpyDeviceToHost, p->diag_stream));
    PHIP(hipStreamSynchronize(p->diag_stream));
    const double N = (double)s.g.nnodes;
    if (k) *k = 0.5 * sums[3] / N;
    if (omega) *omega = 0.5 * sums[6] / N;
    if (rho) PHIP(hipMemcpy(rho, p->d_rho, s.g.nnodes * sizeof(double), hipMemcpyDeviceToHost));
    if (u) PHIP(hipMemcpy(u, p->d_u, 3ull * s.g.nnodes * sizeof(double), hipMemcpyDeviceToHost));
    if (flag) return pfail(KBC_EUNSTABLE, "the box's state is not finite (its run diverged)");
    return KBC_OK;
}

int kbc_pool_release(kbc_pool_handle p, int32_t slot)
{
    if (int r = check_slot(p, slot)) return r;
    Slot& s = p->slots[slot];
    if (s.last) PHIP(hipEventSynchronize(s.last->e));
    if (s.t < s.target) {
        // cancelled while unfinished: no later batch may still refer to it
        PHIP(hipStreamSynchronize(p->stream));
    }
    PHIP(hipStreamSynchronize(p->diag_stream));
    p->arena.release(s.off, s.bytes);
    s = Slot();
    return KBC_OK;
}

int kbc_pool_sync(kbc_pool_handle p)
{
    if (int r = check_pool(p)) return r;
    PHIP(hipSetDevice(p->device));
    PHIP(hipStreamSynchronize(p->stream));
    tuner_collect(p, true);
    return KBC_OK;
}

int kbc_pool_info(kbc_pool_handle p, size_t* bytes_used, int32_t* boxes, int32_t* block, int32_t* grid,
                  int32_t* sub, int32_t* tuning)
{
    if (int r = check_pool(p)) return r;
    int32_t n = 0;
    for (auto& s : p->slots) n += s.used ? 1 : 0;
    if (bytes_used) *bytes_used = p->arena.used();
    if (boxes) *boxes = n;
    if (block) *block = p->cfg.block;
    if (grid) *grid = p->cfg.grid;
    if (sub) *sub = p->cfg.sub;
    if (tuning) *tuning = p->tuning ? 1 : 0;
    return KBC_OK;
}

int kbc_pool_set_launch(kbc_pool_handle p, int32_t block, int32_t grid, int32_t sub)
{
    if (int r = check_pool(p)) return r;
    if (block < 64 || block > kPoolMaxBlock || block % 64 || grid < 0 || sub < 1 || sub > 64)
        return pfail(KBC_EINVAL, "block must be 64..512 in steps of 64, grid >= 0, sub in 1..64");
    tuner_collect(p, true);
    p->cfg = LaunchCfg{block, grid, sub};
    p->fixed = true;
    p->tuning = false;
    return KBC_OK;
}

}  // extern "C"
