// libvpm host layer: the C ABI declared in include/vpm.h.
//
// Every entry point validates its arguments on the host before it makes any HIP call, then
// launches the kernels on the caller's stream and returns without synchronising.  The only
// state kept across calls is a per-device property cache and one pinned staging buffer for
// the batched work queue (both guarded by a mutex).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/vpm.h"
#include "vpm_internal.h"

namespace {

using vpm::kDtypeF32C;
using vpm::kDtypeF64;

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

size_t elem_size(int32_t dtype) { return dtype == kDtypeF64 ? sizeof(double) : sizeof(float); }

bool dtype_ok(int32_t dtype) { return dtype == kDtypeF64 || dtype == kDtypeF32C; }

// Byte range [lo, hi) covered by a [rows][ld] array of n used items per row.
struct Range {
    uintptr_t lo = 0, hi = 0;
};
Range span(const void* p, int rows, int64_t ld, int64_t n, size_t es) {
    Range r;
    if (!p || n <= 0) return r;
    r.lo = reinterpret_cast<uintptr_t>(p);
    r.hi = r.lo + (size_t(rows - 1) * size_t(ld) + size_t(n)) * es;
    return r;
}
bool overlap(const Range& a, const Range& b) {
    return a.hi > a.lo && b.hi > b.lo && a.lo < b.hi && b.lo < a.hi;
}

vpm_status check_offsets(int32_t n_batch, const int64_t* off) {
    if (!off) return VPM_ERR_NULL;
    if (off[0] != 0) return VPM_ERR_OFFSETS;
    for (int32_t b = 0; b < n_batch; ++b)
        if (off[b + 1] < off[b]) return VPM_ERR_OFFSETS;
    return VPM_OK;
}

vpm_status check_options(const vpm_options& o) {
    if (o.scheme != VPM_STRETCH_TRANSPOSED && o.scheme != VPM_STRETCH_CLASSICAL) return VPM_ERR_ENUM;
    if (o.sigma_rule != VPM_SIGMA_SOURCE && o.sigma_rule != VPM_SIGMA_SYMMETRIC) return VPM_ERR_ENUM;
    if (o.self != 0 && o.self != 1) return VPM_ERR_ENUM;
    if (o.accumulate != 0 && o.accumulate != 1) return VPM_ERR_ENUM;
    if (o.variant < 0 || o.variant > vpm::kNumF32Variants) return VPM_ERR_ENUM;
    if (o.gradient != 0 && o.gradient != 1) return VPM_ERR_ENUM;
    for (int i = 0; i < 2; ++i)
        if (o.reserved[i] != 0) return VPM_ERR_ENUM;
    return VPM_OK;
}

vpm_options default_options() {
    vpm_options o;
    std::memset(&o, 0, sizeof(o));
    return o;
}

vpm_status hip_status(hipError_t e) { return e == hipSuccess ? VPM_OK : VPM_ERR_HIP; }

// ------------------------------------------------------------------ device properties
struct DeviceInfo {
    int cus = 0;
};
std::mutex g_mutex;
std::vector<DeviceInfo> g_devices;

hipError_t device_info(DeviceInfo& out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(g_mutex);
    if (int(g_devices.size()) <= dev) g_devices.resize(dev + 1);
    if (g_devices[dev].cus == 0) {
        int cus = 0;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        g_devices[dev].cus = cus;
    }
    out = g_devices[dev];
    return hipSuccess;
}

// ------------------------------------------------------------------ batched work queue
// Workspace layout: [counter | pad][src_off][tgt_off][items], each part 256-byte aligned.
// The smallest target block over all kernel shapes bounds the number of items.
constexpr int64_t kMinTargetsPerBlock = 128;

struct QueueLayout {
    size_t off_src, off_tgt, off_items, total;
    int64_t max_items;
};
int64_t count_blocks(int32_t n_batch, const int64_t* off, int64_t per_block) {
    int64_t items = 0;
    for (int32_t b = 0; b < n_batch; ++b) items += (off[b + 1] - off[b] + per_block - 1) / per_block;
    return items;
}
QueueLayout queue_layout_items(int32_t n_batch, int64_t items) {
    QueueLayout L;
    L.max_items = items;
    L.off_src = kAlign;
    L.off_tgt = L.off_src + align_up(sizeof(int64_t) * (n_batch + 1));
    L.off_items = L.off_tgt + align_up(sizeof(int64_t) * (n_batch + 1));
    L.total = L.off_items + align_up(sizeof(int2) * size_t(items > 0 ? items : 1));
    return L;
}
QueueLayout queue_layout(int32_t n_batch, const int64_t* tgt_off, int64_t per_block) {
    return queue_layout_items(n_batch, count_blocks(n_batch, tgt_off, per_block));
}

// Adjoint of many sets: the larger of the two queues (source blocks, target blocks).
QueueLayout backward_queue_layout(int32_t n_batch, const int64_t* src_off, const int64_t* tgt_off) {
    const int64_t per = vpm::kBwdWG;
    return queue_layout_items(n_batch, std::max(count_blocks(n_batch, src_off, per),
                                                count_blocks(n_batch, tgt_off, per)));
}

hipError_t stage_and_copy(const std::vector<unsigned char>& blob, void* dst, hipStream_t st);

// Stages the LPT-ordered (set, block) items of the lane sets `lane_off` (cost: lane count x
// loop-set size) with both offset tables into the workspace; returns the item count.
hipError_t stage_queue(int32_t n_batch, const int64_t* src_off, const int64_t* tgt_off, bool lane_is_tgt,
                       int64_t per_block, void* workspace, hipStream_t st, int64_t* n_items) {
    const int64_t* lane = lane_is_tgt ? tgt_off : src_off;
    const int64_t* loop = lane_is_tgt ? src_off : tgt_off;
    struct Item {
        int b, blk;
        int64_t cost;
    };
    std::vector<Item> items;
    for (int32_t b = 0; b < n_batch; ++b) {
        const int64_t nl = lane[b + 1] - lane[b], no = loop[b + 1] - loop[b];
        const int64_t nblk = (nl + per_block - 1) / per_block;
        for (int64_t k = 0; k < nblk; ++k)
            items.push_back({b, int(k), (no + 1) * std::min<int64_t>(per_block, nl - k * per_block)});
    }
    *n_items = int64_t(items.size());
    if (items.empty()) return hipSuccess;
    std::stable_sort(items.begin(), items.end(), [](const Item& x, const Item& y) { return x.cost > y.cost; });
    const QueueLayout L = queue_layout_items(n_batch, int64_t(items.size()));
    std::vector<unsigned char> blob(L.off_items + sizeof(int2) * items.size(), 0);
    std::memcpy(blob.data() + L.off_src, src_off, sizeof(int64_t) * (n_batch + 1));
    std::memcpy(blob.data() + L.off_tgt, tgt_off, sizeof(int64_t) * (n_batch + 1));
    int2* it = reinterpret_cast<int2*>(blob.data() + L.off_items);
    for (size_t i = 0; i < items.size(); ++i) {
        it[i].x = items[i].b;
        it[i].y = items[i].blk;
    }
    return stage_and_copy(blob, workspace, st);
}

// Pinned host staging for the queue, reused across calls; the event of the previous copy
// is waited on before the buffer is rewritten.
struct Staging {
    void* host = nullptr;
    size_t bytes = 0;
    hipEvent_t done = nullptr;
    bool pending = false;
};
Staging g_stage;

hipError_t stage_and_copy(const std::vector<unsigned char>& blob, void* dst, hipStream_t st) {
    std::lock_guard<std::mutex> lock(g_mutex);
    hipError_t e;
    if (g_stage.pending) {
        e = hipEventSynchronize(g_stage.done);
        if (e != hipSuccess) return e;
        g_stage.pending = false;
    }
    if (g_stage.bytes < blob.size()) {
        if (g_stage.host) {
            e = hipHostFree(g_stage.host);
            if (e != hipSuccess) return e;
            g_stage.host = nullptr;
            g_stage.bytes = 0;
        }
        e = hipHostMalloc(&g_stage.host, blob.size(), hipHostMallocDefault);
        if (e != hipSuccess) return e;
        g_stage.bytes = blob.size();
    }
    if (!g_stage.done) {
        e = hipEventCreateWithFlags(&g_stage.done, hipEventDisableTiming);
        if (e != hipSuccess) return e;
    }
    std::memcpy(g_stage.host, blob.data(), blob.size());
    e = hipMemcpyAsync(dst, g_stage.host, blob.size(), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    e = hipEventRecord(g_stage.done, st);
    if (e != hipSuccess) return e;
    g_stage.pending = true;
    return hipSuccess;
}

// ------------------------------------------------------------------ kernel-shape plans
// Tuned FP32C kernel shape per (single set / batched, ceil(log2(targets))) bucket, written by
// vpm_set_plan (the tuner); 0 = not set, then the built-in choice.  Guarded by g_mutex.
constexpr int kPlanBuckets = 40;
int g_plan[2][kPlanBuckets] = {};

int plan_bucket(int64_t n) {
    int b = 0;
    while (b < kPlanBuckets - 1 && (int64_t(1) << b) < n) ++b;
    return b;
}

// 0-based variant for an FP32C launch when the caller leaves opt->variant at 0.  The gradient
// mode has a single shape.
// Built-in choice without a tuned plan (what the tuner picks on MI355X): (1, 256, 4) below 16K
// targets and (1, 512, 2) above for one set; (1, 128, 2) for batches.
int default_variant(bool batched, int64_t n_tgt) {
    if (batched) return 5;
    return n_tgt <= 16384 ? 2 : 7;
}

int choose_variant(const vpm_options& o, bool batched, int64_t n_tgt) {
    if (o.gradient) return vpm::kGradientVariant;
    if (o.variant > 0) return o.variant - 1;
    std::lock_guard<std::mutex> lock(g_mutex);
    const int v = g_plan[batched ? 1 : 0][plan_bucket(n_tgt)];
    return v > 0 ? v - 1 : default_variant(batched, n_tgt);
}

int fwd_mode(const vpm_options& o, bool stretch) {
    if (o.gradient) return vpm::kModeGradient;
    if (!stretch) return vpm::kModeVelocity;
    return o.scheme == VPM_STRETCH_CLASSICAL ? vpm::kModeClassical : vpm::kModeTransposed;
}

int64_t targets_per_block(int32_t dtype, int variant) {
    if (dtype == kDtypeF64) return vpm::kF64TargetsPerBlock;
    return int64_t(vpm::kF32Variants[variant].k) * vpm::kF32Variants[variant].wg;
}

// Source split for one small target set: when there are fewer target blocks than
// kSplitBelow, the sources are cut into chunks (multiples of 256, at least kMinChunk) so that
// about kSplitGoal workgroups run; partial sums go to the workspace.  Depends only on sizes.
constexpr int64_t kSplitBelow = 1024;
constexpr int64_t kSplitGoal = 2048;
constexpr int64_t kMinChunk = 256;

struct SplitPlan {
    int64_t nchunk = 1, chunk = 0;
    size_t bytes = 0;
};
SplitPlan split_plan(int32_t dtype, int variant, int nacc, int64_t n_src, int64_t n_tgt) {
    SplitPlan p;
    p.chunk = n_src;
    const int64_t per_block = targets_per_block(dtype, variant);
    const int64_t tblocks = (n_tgt + per_block - 1) / per_block;
    if (tblocks == 0 || tblocks >= kSplitBelow) return p;
    int64_t want = (kSplitGoal + tblocks - 1) / tblocks;
    const int64_t most = n_src / kMinChunk;
    if (want > most) want = most;
    if (want < 2) return p;
    int64_t chunk = (n_src + want - 1) / want;
    chunk = (chunk + 255) / 256 * 256;
    p.chunk = chunk;
    p.nchunk = (n_src + chunk - 1) / chunk;
    if (p.nchunk < 2) {
        p.nchunk = 1;
        p.chunk = n_src;
        return p;
    }
    p.bytes = align_up(size_t(p.nchunk) * size_t(nacc) * size_t(n_tgt) * sizeof(double));
    return p;
}

// The same split with as many chunks as `bytes` of partial sums hold (none below two).
SplitPlan fit_plan(SplitPlan p, int nacc, int64_t n_src, int64_t n_tgt, size_t bytes) {
    const size_t per_chunk = size_t(nacc) * size_t(n_tgt) * sizeof(double);
    for (int64_t most = per_chunk ? int64_t(bytes / per_chunk) : 0; most >= 2; --most) {
        int64_t chunk = (n_src + most - 1) / most;
        chunk = (chunk + 255) / 256 * 256;
        const int64_t nchunk = (n_src + chunk - 1) / chunk;
        const size_t need = align_up(size_t(nchunk) * per_chunk);
        if (nchunk >= 2 && need <= bytes) {
            p.chunk = chunk;
            p.nchunk = nchunk;
            p.bytes = need;
            return p;
        }
    }
    p.chunk = n_src;
    p.nchunk = 1;
    p.bytes = 0;
    return p;
}

// Adjoint of the classical scheme.  Its pair term S_i . (J Gamma_i) equals the transposed
// term Gamma_i . (J^T S_i) with the target's strength and its stretching seed exchanged, while
// the velocity term and the source strengths are unchanged.  So: the transposed adjoint kernel
// with S in the target-strength slot and Gamma in the seed slot gives every position gradient
// and the source strengths' gradient; the target strengths' gradient is the derivative with
// respect to that seed slot, J^T S (the transposed stretching of a target of strength S),
// which the forward kernel adds.  Self evaluations split the two roles of each particle into
// two launches because its strength differs between them.
vpm_status classical_backward(int32_t dtype, bool sym, bool self, int64_t n_src, int64_t n_tgt, const void* x_src,
                              const void* gamma_src, const void* sigma_src, int64_t ld_src, const void* x_tgt,
                              const void* gamma_tgt, const void* sigma_tgt, int64_t ld_tgt, const void* u_bar,
                              const void* dgamma_bar, void* x_src_bar, void* gamma_src_bar, void* x_tgt_bar,
                              void* gamma_tgt_bar, hipStream_t st) {
    // sources as sources (role B): loop over the targets with S in their strength slot
    vpm::BwdArgs b;
    b.xl = x_src; b.gl = gamma_src; b.sl = sigma_src; b.ubl = nullptr; b.sbl = nullptr;
    b.ldl = ld_src; b.nl = n_src;
    b.xo = x_tgt; b.go = dgamma_bar; b.so = sigma_tgt; b.ubo = u_bar; b.sbo = gamma_tgt;
    b.ldo = ld_tgt; b.no = n_tgt;
    b.xbar = x_src_bar; b.gbar = gamma_src_bar; b.ldg = ld_src; b.self = self ? 1 : 0;
    if (vpm::launch_backward(dtype, false, true, true, sym, b, st) != hipSuccess) return VPM_ERR_HIP;
    // targets as targets (role A): their positions; the strength-slot gradient is dropped
    void* xtb = self ? x_src_bar : x_tgt_bar;
    void* gtb = self ? gamma_src_bar : gamma_tgt_bar;
    if (!xtb) return VPM_OK;
    vpm::BwdArgs a;
    a.xl = x_tgt; a.gl = dgamma_bar; a.sl = sigma_tgt; a.ubl = u_bar; a.sbl = gamma_tgt;
    a.ldl = ld_tgt; a.nl = n_tgt;
    a.xo = x_src; a.go = gamma_src; a.so = sigma_src; a.ubo = nullptr; a.sbo = nullptr;
    a.ldo = ld_src; a.no = n_src;
    a.xbar = xtb; a.gbar = nullptr; a.ldg = self ? ld_src : ld_tgt; a.self = self ? 1 : 0;
    if (vpm::launch_backward(dtype, true, false, true, sym, a, st) != hipSuccess) return VPM_ERR_HIP;
    // target strengths: += J^T S (transposed stretching with S as the target strength)
    vpm::FwdArgs f;
    f.xs = x_src; f.gs = gamma_src; f.ss = sigma_src; f.lds = ld_src;
    f.xt = x_tgt; f.gt = dgamma_bar; f.st = sym ? sigma_tgt : nullptr; f.ldt = ld_tgt;
    f.excl = nullptr; f.u = nullptr; f.dg = gtb; f.grad = nullptr; f.ldo = self ? ld_src : ld_tgt;
    f.src_begin = 0; f.src_end = n_src; f.tgt_begin = 0; f.tgt_end = n_tgt;
    f.self = self ? 1 : 0; f.accumulate = 1; f.classical = 0;
    f.part = nullptr; f.chunk = n_src; f.nchunk = 1;
    vpm_options fo = default_options();
    fo.self = self ? 1 : 0;
    const int variant = choose_variant(fo, false, n_tgt);
    const int mode = fwd_mode(fo, true);
    const int64_t per_block = targets_per_block(dtype, variant);
    const int64_t grid = (n_tgt + per_block - 1) / per_block;
    return hip_status(vpm::launch_pair_fwd(dtype, variant, mode, sym, f, nullptr, int(grid), st));
}

// Persistent adjoint launch over many sets: stages the queue of the lane sets' blocks into
// the workspace and fills the GPU with resident workgroups.
hipError_t backward_batched(int32_t dtype, int32_t n_batch, const int64_t* src_off, const int64_t* tgt_off,
                            bool role_a, bool role_b, bool stretch, bool sym, const vpm::BwdArgs& a,
                            bool lane_is_tgt, void* workspace, hipStream_t st) {
    int64_t n_items = 0;
    hipError_t e = stage_queue(n_batch, src_off, tgt_off, lane_is_tgt, vpm::kBwdWG, workspace, st, &n_items);
    if (e != hipSuccess || n_items == 0) return e;
    DeviceInfo di;
    e = device_info(di);
    if (e != hipSuccess) return e;
    int occ = vpm::backward_occupancy(dtype, role_a, role_b, stretch, sym);
    if (occ < 1) occ = 1;
    int64_t grid = std::min<int64_t>(int64_t(di.cus) * occ, n_items);
    const QueueLayout L = queue_layout_items(n_batch, n_items);
    unsigned char* ws = static_cast<unsigned char*>(workspace);
    vpm::BatchQueue q;
    q.counter = reinterpret_cast<int*>(ws);
    q.items = reinterpret_cast<const int2*>(ws + L.off_items);
    q.src_off = reinterpret_cast<const int64_t*>(ws + L.off_src);
    q.tgt_off = reinterpret_cast<const int64_t*>(ws + L.off_tgt);
    q.n_items = int(n_items);
    return vpm::launch_backward_batched(dtype, role_a, role_b, stretch, sym, a, q, int(grid), lane_is_tgt ? 1 : 0,
                                        st);
}

}  // namespace

extern "C" {

const char* vpm_status_string(int32_t s) {
    switch (s) {
        case VPM_OK: return "ok";
        case VPM_ERR_NULL: return "required pointer is NULL";
        case VPM_ERR_SIZE: return "invalid size or leading dimension";
        case VPM_ERR_DTYPE: return "invalid dtype";
        case VPM_ERR_ENUM: return "invalid option or enum value";
        case VPM_ERR_ALIAS: return "output overlaps another argument";
        case VPM_ERR_OFFSETS: return "invalid batch offsets";
        case VPM_ERR_WORKSPACE: return "workspace missing or too small";
        case VPM_ERR_HIP: return "HIP runtime error";
        case VPM_ERR_INPUT: return "invalid input values";
        case VPM_ERR_UNSUPPORTED: return "combination not supported";
        default: return "unknown status";
    }
}

const char* vpm_version(void) { return "libvpm 0.1 (gfx950)"; }

int32_t vpm_variant_count(void) { return vpm::kNumF32Variants; }

vpm_status vpm_variant_info(int32_t k, int32_t* tpl, int32_t* wg) {
    if (k < 1 || k > vpm::kNumF32Variants) return VPM_ERR_ENUM;
    if (!tpl || !wg) return VPM_ERR_NULL;
    *tpl = vpm::kF32Variants[k - 1].k;
    *wg = vpm::kF32Variants[k - 1].wg;
    return VPM_OK;
}

vpm_status vpm_set_plan(int32_t dtype, int32_t batched, int64_t n_lo, int64_t n_hi, int32_t variant) {
    if (dtype != kDtypeF32C) return VPM_ERR_DTYPE;
    if (batched != 0 && batched != 1) return VPM_ERR_ENUM;
    if (variant < 0 || variant > vpm::kNumF32Variants) return VPM_ERR_ENUM;
    if (n_lo < 0 || n_hi < n_lo) return VPM_ERR_SIZE;
    std::lock_guard<std::mutex> lock(g_mutex);
    for (int b = plan_bucket(n_lo); b <= plan_bucket(n_hi); ++b) g_plan[batched][b] = variant;
    return VPM_OK;
}

int32_t vpm_get_plan(int32_t dtype, int32_t batched, int64_t n) {
    if (dtype != kDtypeF32C || (batched != 0 && batched != 1) || n < 0) return 0;
    vpm_options o = default_options();
    return choose_variant(o, batched == 1, n) + 1;
}

size_t vpm_workspace_size(int32_t dtype, int32_t n_batch, const int64_t* src_off,
                          const int64_t* tgt_off, const vpm_options* opt) {
    if (!dtype_ok(dtype) || n_batch < 1 || !src_off) return 0;
    vpm_options o = opt ? *opt : default_options();
    if (o.self && !tgt_off) tgt_off = src_off;
    if (!tgt_off) return 0;
    if (check_offsets(n_batch, src_off) != VPM_OK || check_offsets(n_batch, tgt_off) != VPM_OK) return 0;
    if (check_options(o) != VPM_OK) return 0;
    if (n_batch == 1) {
        const int variant = choose_variant(o, false, tgt_off[1]);
        const int nacc = o.gradient ? vpm::nacc_of(vpm::kModeGradient) : vpm::nacc_of(vpm::kModeTransposed);
        return split_plan(dtype, variant, nacc, src_off[1], tgt_off[1]).bytes;
    }
    return queue_layout(n_batch, tgt_off, kMinTargetsPerBlock).total;
}

}  // extern "C"

namespace {

// Shared body of vpm_eval_velocity_stretching (grad_out == nullptr, o.gradient == 0) and
// vpm_eval_velocity_gradient (o.gradient == 1).
vpm_status eval_impl(int32_t dtype, int32_t n_batch, const int64_t* src_off, const int64_t* tgt_off,
                     const void* x_src, const void* gamma_src, const void* sigma_src, int64_t ld_src,
                     const void* x_tgt, const void* gamma_tgt, const void* sigma_tgt, int64_t ld_tgt,
                     const int32_t* tgt_exclude, void* u_out, void* dgamma_out, void* grad_out, int64_t ld_out,
                     vpm_options o, void* workspace, size_t ws_bytes, void* stream, bool noalloc = false) {
    if (!dtype_ok(dtype)) return VPM_ERR_DTYPE;
    if (n_batch < 1) return VPM_ERR_SIZE;
    vpm_status s = check_options(o);
    if (s != VPM_OK) return s;
    if (!src_off) return VPM_ERR_NULL;
    s = check_offsets(n_batch, src_off);
    if (s != VPM_OK) return s;
    if (o.self) {
        if (tgt_off && tgt_off != src_off) {
            for (int32_t b = 0; b <= n_batch; ++b)
                if (tgt_off[b] != src_off[b]) return VPM_ERR_OFFSETS;
        }
        tgt_off = src_off;
        if ((x_tgt && x_tgt != x_src) || (gamma_tgt && gamma_tgt != gamma_src) ||
            (sigma_tgt && sigma_tgt != sigma_src))
            return VPM_ERR_ALIAS;
        if (ld_tgt != 0 && ld_tgt != ld_src) return VPM_ERR_SIZE;
        x_tgt = x_src;
        gamma_tgt = gamma_src;
        sigma_tgt = sigma_src;
        ld_tgt = ld_src;
        tgt_exclude = nullptr;
    } else {
        if (!tgt_off) return VPM_ERR_NULL;
        s = check_offsets(n_batch, tgt_off);
        if (s != VPM_OK) return s;
    }
    const int64_t n_src = src_off[n_batch];
    const int64_t n_tgt = tgt_off[n_batch];
    if (n_src > INT32_MAX || n_tgt > INT32_MAX) return VPM_ERR_SIZE;
    if (ld_src < n_src || ld_tgt < n_tgt || ld_out < n_tgt) return VPM_ERR_SIZE;
    if (n_src > 0 && (!x_src || !gamma_src || !sigma_src)) return VPM_ERR_NULL;
    if (n_tgt > 0 && (!x_tgt || !u_out)) return VPM_ERR_NULL;
    const bool stretch = dgamma_out != nullptr;
    if (stretch && !gamma_tgt) return VPM_ERR_NULL;
    if (o.gradient && n_tgt > 0 && (!stretch || !grad_out)) return VPM_ERR_NULL;
    const bool sym = o.sigma_rule == VPM_SIGMA_SYMMETRIC;
    if (sym && n_tgt > 0 && !sigma_tgt) return VPM_ERR_NULL;

    const size_t es = elem_size(dtype);
    const Range ru = span(u_out, 3, ld_out, n_tgt, es);
    const Range rd = span(dgamma_out, 3, ld_out, n_tgt, es);
    const Range rj = span(o.gradient ? grad_out : nullptr, 9, ld_out, n_tgt, es);
    const Range ins[7] = {span(x_src, 3, ld_src, n_src, es),   span(gamma_src, 3, ld_src, n_src, es),
                          span(sigma_src, 1, ld_src, n_src, es), span(x_tgt, 3, ld_tgt, n_tgt, es),
                          span(gamma_tgt, 3, ld_tgt, n_tgt, es), span(sigma_tgt, 1, ld_tgt, n_tgt, es),
                          span(tgt_exclude, 1, n_tgt, n_tgt, sizeof(int32_t))};
    for (const Range& r : ins)
        if (overlap(ru, r) || overlap(rd, r) || overlap(rj, r)) return VPM_ERR_ALIAS;
    if (overlap(ru, rd) || overlap(ru, rj) || overlap(rd, rj)) return VPM_ERR_ALIAS;

    const int variant = choose_variant(o, n_batch > 1, n_tgt);
    if (workspace && ws_bytes > 0) {
        const Range rw = span(workspace, 1, int64_t(ws_bytes), int64_t(ws_bytes), 1);
        if (overlap(rw, ru) || overlap(rw, rd) || overlap(rw, rj)) return VPM_ERR_ALIAS;
        for (const Range& r : ins)
            if (overlap(rw, r)) return VPM_ERR_ALIAS;
    }
    QueueLayout L{};
    if (n_batch > 1) {
        L = queue_layout(n_batch, tgt_off, kMinTargetsPerBlock);
        if (!workspace) return VPM_ERR_WORKSPACE;
        if (ws_bytes < L.total) return VPM_ERR_WORKSPACE;
    }
    if (n_tgt == 0) return VPM_OK;

    // ---- launch (first HIP call)
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (noalloc) {
        // the source-split partials go to the library's own scratch array
        if (vpm::noalloc_scratch(&workspace) != hipSuccess) return VPM_ERR_HIP;
        ws_bytes = vpm::kNoAllocScratchBytes;
    }
    vpm::FwdArgs a;
    a.xs = x_src;
    a.gs = gamma_src;
    a.ss = sigma_src;
    a.lds = ld_src;
    a.xt = x_tgt;
    a.gt = stretch ? gamma_tgt : nullptr;
    a.st = sym ? sigma_tgt : nullptr;
    a.ldt = ld_tgt;
    a.excl = tgt_exclude;
    a.u = u_out;
    a.dg = dgamma_out;
    a.grad = o.gradient ? grad_out : nullptr;
    a.ldo = ld_out;
    a.src_begin = 0;
    a.src_end = n_src;
    a.tgt_begin = 0;
    a.tgt_end = n_tgt;
    a.self = o.self;
    a.accumulate = o.accumulate;
    a.classical = o.scheme == VPM_STRETCH_CLASSICAL;
    a.part = nullptr;
    a.chunk = n_src;
    a.nchunk = 1;
    const int mode = fwd_mode(o, stretch);
    const int64_t per_block = targets_per_block(dtype, variant);

    if (n_batch == 1) {
        SplitPlan sp = split_plan(dtype, variant, vpm::nacc_of(mode), n_src, n_tgt);
        if (noalloc && sp.nchunk > 1 && sp.bytes > ws_bytes)
            sp = fit_plan(sp, vpm::nacc_of(mode), n_src, n_tgt, ws_bytes);
        if (sp.nchunk > 1 && workspace && ws_bytes >= sp.bytes) {
            a.part = static_cast<double*>(workspace);
            a.chunk = sp.chunk;
            a.nchunk = int32_t(sp.nchunk);
        }
        const int64_t grid = (n_tgt + per_block - 1) / per_block;
        return hip_status(vpm::launch_pair_fwd(dtype, variant, mode, sym, a, nullptr, int(grid), st));
    }

    // Batched: LPT-ordered (set, block) items, staged into the workspace with the counter.
    struct Item {
        int b, blk;
        int64_t cost;
    };
    std::vector<Item> items;
    for (int32_t b = 0; b < n_batch; ++b) {
        const int64_t nt = tgt_off[b + 1] - tgt_off[b];
        const int64_t ns = src_off[b + 1] - src_off[b];
        const int64_t nblk = (nt + per_block - 1) / per_block;
        for (int64_t k = 0; k < nblk; ++k) {
            const int64_t tk = std::min<int64_t>(per_block, nt - k * per_block);
            items.push_back({b, int(k), (ns + 1) * tk});
        }
    }
    if (items.empty()) return VPM_OK;
    std::stable_sort(items.begin(), items.end(), [](const Item& x, const Item& y) { return x.cost > y.cost; });
    std::vector<unsigned char> blob(L.off_items + sizeof(int2) * items.size(), 0);
    std::memcpy(blob.data() + L.off_src, src_off, sizeof(int64_t) * (n_batch + 1));
    std::memcpy(blob.data() + L.off_tgt, tgt_off, sizeof(int64_t) * (n_batch + 1));
    int2* it = reinterpret_cast<int2*>(blob.data() + L.off_items);
    for (size_t i = 0; i < items.size(); ++i) {
        it[i].x = items[i].b;
        it[i].y = items[i].blk;
    }
    hipError_t e = stage_and_copy(blob, workspace, st);
    if (e != hipSuccess) return VPM_ERR_HIP;
    DeviceInfo di;
    e = device_info(di);
    if (e != hipSuccess) return VPM_ERR_HIP;
    int occ = vpm::pair_fwd_occupancy(dtype, variant, mode, sym, true);
    if (occ < 1) occ = 1;
    int64_t grid = int64_t(di.cus) * occ;
    if (grid > int64_t(items.size())) grid = int64_t(items.size());
    unsigned char* ws = static_cast<unsigned char*>(workspace);
    vpm::BatchQueue q;
    q.counter = reinterpret_cast<int*>(ws);
    q.items = reinterpret_cast<const int2*>(ws + L.off_items);
    q.src_off = reinterpret_cast<const int64_t*>(ws + L.off_src);
    q.tgt_off = reinterpret_cast<const int64_t*>(ws + L.off_tgt);
    q.n_items = int(items.size());
    return hip_status(vpm::launch_pair_fwd(dtype, variant, mode, sym, a, &q, int(grid), st));
}

}  // namespace

extern "C" {

vpm_status vpm_eval_velocity_stretching(int32_t dtype, int32_t n_batch, const int64_t* src_off,
                                        const int64_t* tgt_off, const void* x_src,
                                        const void* gamma_src, const void* sigma_src,
                                        int64_t ld_src, const void* x_tgt, const void* gamma_tgt,
                                        const void* sigma_tgt, int64_t ld_tgt,
                                        const int32_t* tgt_exclude, void* u_out, void* dgamma_out,
                                        int64_t ld_out, const vpm_options* opt, void* workspace,
                                        size_t ws_bytes, void* stream) {
    vpm_options o = opt ? *opt : default_options();
    if (o.gradient != 0) return VPM_ERR_ENUM;
    return eval_impl(dtype, n_batch, src_off, tgt_off, x_src, gamma_src, sigma_src, ld_src, x_tgt, gamma_tgt,
                     sigma_tgt, ld_tgt, tgt_exclude, u_out, dgamma_out, nullptr, ld_out, o, workspace, ws_bytes,
                     stream);
}

vpm_status vpm_eval_velocity_stretching_noalloc(int32_t dtype, int32_t n_batch, const int64_t* src_off,
                                                const int64_t* tgt_off, const void* x_src, const void* gamma_src,
                                                const void* sigma_src, int64_t ld_src, const void* x_tgt,
                                                const void* gamma_tgt, const void* sigma_tgt, int64_t ld_tgt,
                                                const int32_t* tgt_exclude, void* u_out, void* dgamma_out,
                                                int64_t ld_out, const vpm_options* opt, void* stream) {
    if (!dtype_ok(dtype)) return VPM_ERR_DTYPE;
    if (n_batch < 1) return VPM_ERR_SIZE;
    if (n_batch != 1) return VPM_ERR_UNSUPPORTED;  // the batched queue is staged from host memory
    vpm_options o = opt ? *opt : default_options();
    if (o.gradient != 0) return VPM_ERR_ENUM;
    return eval_impl(dtype, n_batch, src_off, tgt_off, x_src, gamma_src, sigma_src, ld_src, x_tgt, gamma_tgt,
                     sigma_tgt, ld_tgt, tgt_exclude, u_out, dgamma_out, nullptr, ld_out, o, nullptr, 0, stream, true);
}

size_t vpm_noalloc_scratch_bytes(void) { return vpm::kNoAllocScratchBytes; }

vpm_status vpm_eval_velocity_gradient(int32_t dtype, int32_t n_batch, const int64_t* src_off,
                                      const int64_t* tgt_off, const void* x_src, const void* gamma_src,
                                      const void* sigma_src, int64_t ld_src, const void* x_tgt,
                                      const void* gamma_tgt, const void* sigma_tgt, int64_t ld_tgt,
                                      const int32_t* tgt_exclude, void* u_out, void* dgamma_out,
                                      void* grad_out, int64_t ld_out, const vpm_options* opt,
                                      void* workspace, size_t ws_bytes, void* stream) {
    vpm_options o = opt ? *opt : default_options();
    if (o.gradient != 0 && o.gradient != 1) return VPM_ERR_ENUM;
    o.gradient = 1;
    const vpm_status s = check_options(o);  // the caller's fields, before the shape is fixed
    if (s != VPM_OK) return s;
    o.variant = 0;
    return eval_impl(dtype, n_batch, src_off, tgt_off, x_src, gamma_src, sigma_src, ld_src, x_tgt, gamma_tgt,
                     sigma_tgt, ld_tgt, tgt_exclude, u_out, dgamma_out, grad_out, ld_out, o, workspace, ws_bytes,
                     stream);
}

vpm_status vpm_sgs_vreman(int32_t dtype, int64_t n, const void* grad, const void* sigma, int64_t ld, double c_v,
                          void* nu_t_out, void* stream) {
    if (!dtype_ok(dtype)) return VPM_ERR_DTYPE;
    if (n < 0 || ld < n || n > INT32_MAX) return VPM_ERR_SIZE;
    if (!(c_v >= 0.0) || c_v > 1e30) return VPM_ERR_SIZE;
    if (n == 0) return VPM_OK;
    if (!grad || !sigma || !nu_t_out) return VPM_ERR_NULL;
    const size_t es = elem_size(dtype);
    const Range ro = span(nu_t_out, 1, ld, n, es);
    if (overlap(ro, span(grad, 9, ld, n, es)) || overlap(ro, span(sigma, 1, ld, n, es))) return VPM_ERR_ALIAS;
    return hip_status(vpm::launch_vreman(dtype, n, grad, ld, sigma, c_v, nu_t_out, static_cast<hipStream_t>(stream)));
}

size_t vpm_diffusion_workspace_size(int32_t dtype, int32_t n_batch, const int64_t* off) {
    if (!dtype_ok(dtype) || n_batch < 1 || check_offsets(n_batch, off) != VPM_OK) return 0;
    size_t most = 0;
    for (int32_t b = 0; b < n_batch; ++b)
        if (off[b + 1] > off[b]) most = std::max(most, vpm::pse_workspace(off[b + 1] - off[b], dtype));
    return most;
}

vpm_status vpm_eval_diffusion(int32_t dtype, int32_t n_batch, const int64_t* off, const void* x,
                              const void* gamma, const void* sigma, const void* vol, const void* nu_t,
                              int64_t ld, double nu, void* dgamma_out, int64_t ld_out, int32_t accumulate,
                              void* workspace, size_t ws_bytes, void* stream) {
    if (!dtype_ok(dtype)) return VPM_ERR_DTYPE;
    if (n_batch < 1) return VPM_ERR_SIZE;
    vpm_status s = check_offsets(n_batch, off);
    if (s != VPM_OK) return s;
    const int64_t n = off[n_batch];
    if (n > INT32_MAX || ld < n || ld_out < n) return VPM_ERR_SIZE;
    if (!(nu >= 0.0) || nu > 1e30) return VPM_ERR_SIZE;
    if (accumulate != 0 && accumulate != 1) return VPM_ERR_ENUM;
    if (n == 0) return VPM_OK;
    if (!x || !gamma || !sigma || !vol || !dgamma_out) return VPM_ERR_NULL;
    const size_t need = vpm_diffusion_workspace_size(dtype, n_batch, off);
    if (need == 0) return VPM_ERR_SIZE;
    if (!workspace || ws_bytes < need) return VPM_ERR_WORKSPACE;
    const size_t es = elem_size(dtype);
    const Range rd = span(dgamma_out, 3, ld_out, n, es);
    const Range rw = span(workspace, 1, int64_t(ws_bytes), int64_t(ws_bytes), 1);
    const Range ins[5] = {span(x, 3, ld, n, es), span(gamma, 3, ld, n, es), span(sigma, 1, ld, n, es),
                          span(vol, 1, ld, n, es), span(nu_t, 1, ld, n, es)};
    for (const Range& r : ins)
        if (overlap(rd, r) || overlap(rw, r)) return VPM_ERR_ALIAS;
    if (overlap(rd, rw)) return VPM_ERR_ALIAS;
    hipStream_t st = static_cast<hipStream_t>(stream);
    // the sets run one after the other on the stream and reuse the workspace
    for (int32_t b = 0; b < n_batch; ++b) {
        if (off[b + 1] == off[b]) continue;
        hipError_t e = vpm::launch_pse(dtype, off[b], off[b + 1], x, gamma, sigma, vol, nu_t, ld, nu, dgamma_out,
                                       ld_out, accumulate, workspace, st);
        if (e != hipSuccess) return VPM_ERR_HIP;
    }
    return VPM_OK;
}

vpm_status vpm_eval_segments(int32_t dtype, int64_t n_seg, const void* a, const void* b,
                             const void* gamma_seg, int64_t ld_seg, double core_radius,
                             int32_t vatistas_n, int64_t n_tgt, const void* x_tgt, int64_t ld_tgt,
                             void* u_out, int64_t ld_out, int32_t accumulate, void* stream) {
    if (!dtype_ok(dtype)) return VPM_ERR_DTYPE;
    if (n_seg < 0 || n_tgt < 0 || ld_seg < n_seg || ld_tgt < n_tgt || ld_out < n_tgt) return VPM_ERR_SIZE;
    if (n_seg > INT32_MAX || n_tgt > INT32_MAX) return VPM_ERR_SIZE;
    if (n_seg > 0 && (!a || !b || !gamma_seg)) return VPM_ERR_NULL;
    if (n_tgt > 0 && (!x_tgt || !u_out)) return VPM_ERR_NULL;
    if (!(core_radius >= 0.0) || core_radius > 1e30) return VPM_ERR_SIZE;
    if (vatistas_n < 1 || vatistas_n > 16) return VPM_ERR_ENUM;
    if (accumulate != 0 && accumulate != 1) return VPM_ERR_ENUM;
    const size_t es = elem_size(dtype);
    const Range ru = span(u_out, 3, ld_out, n_tgt, es);
    const Range ins[4] = {span(a, 3, ld_seg, n_seg, es), span(b, 3, ld_seg, n_seg, es),
                          span(gamma_seg, 1, ld_seg, n_seg, es), span(x_tgt, 3, ld_tgt, n_tgt, es)};
    for (const Range& r : ins)
        if (overlap(ru, r)) return VPM_ERR_ALIAS;
    if (n_tgt == 0) return VPM_OK;
    vpm::SegArgs s{};
    s.a = a;
    s.b = b;
    s.gam = gamma_seg;
    s.ld_seg = ld_seg;
    s.n_seg = n_seg;
    s.rc = core_radius;
    s.vn = vatistas_n;
    s.xt = x_tgt;
    s.ldt = ld_tgt;
    s.n_tgt = n_tgt;
    s.u = u_out;
    s.ldo = ld_out;
    s.accumulate = accumulate;
    return hip_status(vpm::launch_segments(dtype, s, static_cast<hipStream_t>(stream)));
}

vpm_status vpm_eval_segments_gradient(int32_t dtype, int64_t n_seg, const void* a, const void* b,
                                      const void* gamma_seg, int64_t ld_seg, double core_radius,
                                      int32_t vatistas_n, int64_t n_tgt, const void* x_tgt, const void* gamma_tgt,
                                      int64_t ld_tgt, int32_t scheme, void* u_out, void* grad_out,
                                      void* dgamma_out, int64_t ld_out, int32_t accumulate, void* stream) {
    if (!dtype_ok(dtype)) return VPM_ERR_DTYPE;
    if (n_seg < 0 || n_tgt < 0 || ld_seg < n_seg || ld_tgt < n_tgt || ld_out < n_tgt) return VPM_ERR_SIZE;
    if (n_seg > INT32_MAX || n_tgt > INT32_MAX) return VPM_ERR_SIZE;
    if (n_seg > 0 && (!a || !b || !gamma_seg)) return VPM_ERR_NULL;
    if (n_tgt > 0 && ((!u_out && !grad_out && !dgamma_out) || !x_tgt)) return VPM_ERR_NULL;
    if (dgamma_out && n_tgt > 0 && !gamma_tgt) return VPM_ERR_NULL;
    if (!(core_radius >= 0.0) || core_radius > 1e30) return VPM_ERR_SIZE;
    if (vatistas_n < 1 || vatistas_n > 16) return VPM_ERR_ENUM;
    if (scheme != VPM_STRETCH_TRANSPOSED && scheme != VPM_STRETCH_CLASSICAL) return VPM_ERR_ENUM;
    if (accumulate != 0 && accumulate != 1) return VPM_ERR_ENUM;
    const size_t es = elem_size(dtype);
    const Range outs[3] = {u_out ? span(u_out, 3, ld_out, n_tgt, es) : Range{},
                           grad_out ? span(grad_out, 9, ld_out, n_tgt, es) : Range{},
                           dgamma_out ? span(dgamma_out, 3, ld_out, n_tgt, es) : Range{}};
    const Range ins[5] = {span(a, 3, ld_seg, n_seg, es), span(b, 3, ld_seg, n_seg, es),
                          span(gamma_seg, 1, ld_seg, n_seg, es), span(x_tgt, 3, ld_tgt, n_tgt, es),
                          dgamma_out ? span(gamma_tgt, 3, ld_tgt, n_tgt, es) : Range{}};
    for (int i = 0; i < 3; ++i) {
        for (const Range& r : ins)
            if (overlap(outs[i], r)) return VPM_ERR_ALIAS;
        for (int j = i + 1; j < 3; ++j)
            if (overlap(outs[i], outs[j])) return VPM_ERR_ALIAS;
    }
    if (n_tgt == 0) return VPM_OK;
    vpm::SegArgs s{};
    s.a = a;
    s.b = b;
    s.gam = gamma_seg;
    s.ld_seg = ld_seg;
    s.n_seg = n_seg;
    s.rc = core_radius;
    s.vn = vatistas_n;
    s.xt = x_tgt;
    s.ldt = ld_tgt;
    s.n_tgt = n_tgt;
    s.u = u_out;
    s.ldo = ld_out;
    s.accumulate = accumulate;
    s.gt = dgamma_out ? gamma_tgt : nullptr;
    s.grad = grad_out;
    s.dg = dgamma_out;
    s.classical = scheme == VPM_STRETCH_CLASSICAL;
    return hip_status(vpm::launch_segments_gradient(dtype, s, static_cast<hipStream_t>(stream)));
}

vpm_status vpm_segments_backward(int32_t dtype, int64_t n_seg, const void* a, const void* b,
                                 const void* gamma_seg, int64_t ld_seg, double core_radius, int32_t vatistas_n,
                                 int64_t n_tgt, const void* x_tgt, const void* gamma_tgt, int64_t ld_tgt,
                                 int32_t scheme, const void* u_bar, const void* dgamma_bar, int64_t ld_bar,
                                 void* x_bar, void* gamma_bar, int64_t ld_grad, void* stream) {
    if (!dtype_ok(dtype)) return VPM_ERR_DTYPE;
    if (n_seg < 0 || n_tgt < 0 || ld_seg < n_seg || ld_tgt < n_tgt || ld_bar < n_tgt || ld_grad < n_tgt)
        return VPM_ERR_SIZE;
    if (n_seg > INT32_MAX || n_tgt > INT32_MAX) return VPM_ERR_SIZE;
    if (n_seg > 0 && (!a || !b || !gamma_seg)) return VPM_ERR_NULL;
    if (n_tgt > 0) {
        if (!x_tgt || !x_bar || (!u_bar && !dgamma_bar)) return VPM_ERR_NULL;
        if (dgamma_bar && (!gamma_tgt || !gamma_bar)) return VPM_ERR_NULL;
    }
    if (!(core_radius >= 0.0) || core_radius > 1e30) return VPM_ERR_SIZE;
    if (vatistas_n < 1 || vatistas_n > 16) return VPM_ERR_ENUM;
    if (scheme != VPM_STRETCH_TRANSPOSED && scheme != VPM_STRETCH_CLASSICAL) return VPM_ERR_ENUM;
    const size_t es = elem_size(dtype);
    const Range outs[2] = {span(x_bar, 3, ld_grad, n_tgt, es),
                           dgamma_bar ? span(gamma_bar, 3, ld_grad, n_tgt, es) : Range{}};
    const Range ins[7] = {span(a, 3, ld_seg, n_seg, es), span(b, 3, ld_seg, n_seg, es),
                          span(gamma_seg, 1, ld_seg, n_seg, es), span(x_tgt, 3, ld_tgt, n_tgt, es),
                          dgamma_bar ? span(gamma_tgt, 3, ld_tgt, n_tgt, es) : Range{},
                          span(u_bar, 3, ld_bar, n_tgt, es), span(dgamma_bar, 3, ld_bar, n_tgt, es)};
    for (const Range& o : outs)
        for (const Range& r : ins)
            if (overlap(o, r)) return VPM_ERR_ALIAS;
    if (overlap(outs[0], outs[1])) return VPM_ERR_ALIAS;
    if (n_tgt == 0) return VPM_OK;
    vpm::SegArgs s{};
    s.a = a;
    s.b = b;
    s.gam = gamma_seg;
    s.ld_seg = ld_seg;
    s.n_seg = n_seg;
    s.rc = core_radius;
    s.vn = vatistas_n;
    s.xt = x_tgt;
    s.ldt = ld_tgt;
    s.n_tgt = n_tgt;
    s.ldo = ld_grad;
    s.gt = dgamma_bar ? gamma_tgt : nullptr;
    s.classical = scheme == VPM_STRETCH_CLASSICAL;
    s.ub = u_bar;
    s.db = dgamma_bar;
    s.ldb = ld_bar;
    s.xb = x_bar;
    s.gb = dgamma_bar ? gamma_bar : nullptr;
    return hip_status(vpm::launch_segments_vjp(dtype, s, static_cast<hipStream_t>(stream)));
}

size_t vpm_fmm_workspace_size(int32_t dtype, int64_t n, int32_t level, int32_t order) {
    if (!dtype_ok(dtype) || n < 0 || n > INT32_MAX / 2 || level < 0 || level > 10 || order < 1 || order > 20)
        return 0;
    return vpm::fmm_workspace(n, level, order, dtype);
}

vpm_status vpm_fmm_eval(int32_t dtype, int64_t n, const void* x, const void* gamma, const void* sigma, int64_t ld,
                        int32_t level, int32_t order, int32_t scheme, void* u_out, void* dgamma_out, void* grad_out,
                        int64_t ld_out, void* workspace, size_t ws_bytes, void* stream) {
    if (!dtype_ok(dtype)) return VPM_ERR_DTYPE;
    if (n < 0 || n > INT32_MAX / 2 || ld < n || ld_out < n) return VPM_ERR_SIZE;
    if (level < 0 || level > 10 || order < 1 || order > 20) return VPM_ERR_ENUM;
    if (scheme != VPM_STRETCH_TRANSPOSED && scheme != VPM_STRETCH_CLASSICAL) return VPM_ERR_ENUM;
    if (n > 0 && (!x || !gamma || !sigma || !u_out || !dgamma_out)) return VPM_ERR_NULL;
    const size_t es = elem_size(dtype);
    const Range ru = span(u_out, 3, ld_out, n, es), rd = span(dgamma_out, 3, ld_out, n, es);
    const Range rg = span(grad_out, 9, ld_out, n, es);
    const Range ins[3] = {span(x, 3, ld, n, es), span(gamma, 3, ld, n, es), span(sigma, 1, ld, n, es)};
    for (const Range& r : ins)
        if (overlap(ru, r) || overlap(rd, r) || overlap(rg, r)) return VPM_ERR_ALIAS;
    if (overlap(ru, rd) || overlap(ru, rg) || overlap(rd, rg)) return VPM_ERR_ALIAS;
    if (n == 0) return VPM_OK;
    const size_t need = vpm::fmm_workspace(n, level, order, dtype);
    if (!workspace || ws_bytes < need) return VPM_ERR_WORKSPACE;
    const Range rw = span(workspace, 1, int64_t(need), int64_t(need), 1);
    for (const Range& r : ins)
        if (overlap(rw, r)) return VPM_ERR_ALIAS;
    if (overlap(rw, ru) || overlap(rw, rd) || overlap(rw, rg)) return VPM_ERR_ALIAS;
    return hip_status(vpm::launch_fmm(dtype, n, x, gamma, sigma, ld, level, order, scheme == VPM_STRETCH_CLASSICAL,
                                      u_out, dgamma_out, grad_out, ld_out, workspace,
                                      static_cast<hipStream_t>(stream)));
}

vpm_status vpm_backward(int32_t dtype, int32_t n_batch, const int64_t* src_off,
                        const int64_t* tgt_off, const void* x_src, const void* gamma_src,
                        const void* sigma_src, int64_t ld_src, const void* x_tgt,
                        const void* gamma_tgt, const void* sigma_tgt, int64_t ld_tgt,
                        const void* u_bar, const void* dgamma_bar, void* x_src_bar,
                        void* gamma_src_bar, void* x_tgt_bar, void* gamma_tgt_bar,
                        const vpm_options* opt, void* workspace, size_t ws_bytes, void* stream) {
    if (!dtype_ok(dtype)) return VPM_ERR_DTYPE;
    if (n_batch < 1) return VPM_ERR_SIZE;
    vpm_options o = opt ? *opt : default_options();
    vpm_status s = check_options(o);
    if (s != VPM_OK) return s;
    if (!src_off) return VPM_ERR_NULL;
    s = check_offsets(n_batch, src_off);
    if (s != VPM_OK) return s;
    // Gradients are always accumulated (+=); opt->accumulate is not consulted.
    if (o.self) {
        if (tgt_off && tgt_off != src_off) {
            for (int32_t b = 0; b <= n_batch; ++b)
                if (tgt_off[b] != src_off[b]) return VPM_ERR_OFFSETS;
        }
        if ((x_tgt && x_tgt != x_src) || (gamma_tgt && gamma_tgt != gamma_src) ||
            (sigma_tgt && sigma_tgt != sigma_src))
            return VPM_ERR_ALIAS;
        if (x_tgt_bar || gamma_tgt_bar) return VPM_ERR_ALIAS;
        if (ld_tgt != 0 && ld_tgt != ld_src) return VPM_ERR_SIZE;
        tgt_off = src_off;
        x_tgt = x_src;
        gamma_tgt = gamma_src;
        sigma_tgt = sigma_src;
        ld_tgt = ld_src;
    } else {
        if (!tgt_off) return VPM_ERR_NULL;
        s = check_offsets(n_batch, tgt_off);
        if (s != VPM_OK) return s;
    }
    const int64_t n_src = src_off[n_batch];
    const int64_t n_tgt = tgt_off[n_batch];
    if (n_src > INT32_MAX || n_tgt > INT32_MAX) return VPM_ERR_SIZE;
    if (ld_src < n_src || ld_tgt < n_tgt) return VPM_ERR_SIZE;
    const bool stretch = dgamma_bar != nullptr;
    const bool sym = o.sigma_rule == VPM_SIGMA_SYMMETRIC;
    if (n_src > 0 && (!x_src || !gamma_src || !sigma_src || !x_src_bar || !gamma_src_bar)) return VPM_ERR_NULL;
    if (n_tgt > 0 && (!x_tgt || !u_bar)) return VPM_ERR_NULL;
    if (n_tgt > 0 && stretch && !gamma_tgt) return VPM_ERR_NULL;
    if (n_tgt > 0 && sym && !sigma_tgt) return VPM_ERR_NULL;
    const bool want_tgt = !o.self && (x_tgt_bar || gamma_tgt_bar);
    if (want_tgt && (!x_tgt_bar || (stretch && !gamma_tgt_bar))) return VPM_ERR_NULL;

    const size_t es = elem_size(dtype);
    const Range outs[4] = {span(x_src_bar, 3, ld_src, n_src, es), span(gamma_src_bar, 3, ld_src, n_src, es),
                           span(x_tgt_bar, 3, ld_tgt, n_tgt, es), span(gamma_tgt_bar, 3, ld_tgt, n_tgt, es)};
    const Range ins[8] = {span(x_src, 3, ld_src, n_src, es),    span(gamma_src, 3, ld_src, n_src, es),
                          span(sigma_src, 1, ld_src, n_src, es),  span(x_tgt, 3, ld_tgt, n_tgt, es),
                          span(gamma_tgt, 3, ld_tgt, n_tgt, es),  span(sigma_tgt, 1, ld_tgt, n_tgt, es),
                          span(u_bar, 3, ld_tgt, n_tgt, es),      span(dgamma_bar, 3, ld_tgt, n_tgt, es)};
    for (int i = 0; i < 4; ++i) {
        for (const Range& r : ins)
            if (overlap(outs[i], r)) return VPM_ERR_ALIAS;
        for (int j = i + 1; j < 4; ++j)
            if (overlap(outs[i], outs[j])) return VPM_ERR_ALIAS;
    }
    const bool classical = o.scheme == VPM_STRETCH_CLASSICAL && stretch;
    if (n_batch > 1 && !classical) {
        const QueueLayout L = backward_queue_layout(n_batch, src_off, tgt_off);
        if (!workspace || ws_bytes < L.total) return VPM_ERR_WORKSPACE;
        const Range rw = span(workspace, 1, int64_t(ws_bytes), int64_t(ws_bytes), 1);
        for (int i = 0; i < 4; ++i)
            if (overlap(rw, outs[i])) return VPM_ERR_ALIAS;
        for (const Range& r : ins)
            if (overlap(rw, r)) return VPM_ERR_ALIAS;
    }
    if (n_src == 0 && n_tgt == 0) return VPM_OK;

    hipStream_t st = static_cast<hipStream_t>(stream);
    if (classical) {
        // one set after another (the composition runs three launches per set)
        auto sh = [es](const void* q, int64_t off) -> const void* {
            return q ? static_cast<const unsigned char*>(q) + size_t(off) * es : nullptr;
        };
        auto shm = [es](void* q, int64_t off) -> void* {
            return q ? static_cast<unsigned char*>(q) + size_t(off) * es : nullptr;
        };
        for (int32_t b = 0; b < n_batch; ++b) {
            const int64_t s0 = src_off[b], t0 = tgt_off[b];
            const int64_t ns = src_off[b + 1] - s0, nt = tgt_off[b + 1] - t0;
            if (ns == 0 && nt == 0) continue;
            const vpm_status r = classical_backward(
                dtype, sym, o.self != 0, ns, nt, sh(x_src, s0), sh(gamma_src, s0), sh(sigma_src, s0), ld_src,
                sh(x_tgt, t0), sh(gamma_tgt, t0), sh(sigma_tgt, t0), ld_tgt, sh(u_bar, t0), sh(dgamma_bar, t0),
                shm(x_src_bar, s0), shm(gamma_src_bar, s0), want_tgt ? shm(x_tgt_bar, t0) : nullptr,
                want_tgt ? shm(gamma_tgt_bar, t0) : nullptr, st);
            if (r != VPM_OK) return r;
        }
        return VPM_OK;
    }
    vpm::BwdArgs a;
    if (o.self) {
        a.xl = x_src; a.gl = gamma_src; a.sl = sigma_src; a.ubl = u_bar; a.sbl = dgamma_bar;
        a.ldl = ld_src; a.nl = n_src;
        a.xo = x_src; a.go = gamma_src; a.so = sigma_src; a.ubo = u_bar; a.sbo = dgamma_bar;
        a.ldo = ld_src; a.no = n_src;
        a.xbar = x_src_bar; a.gbar = gamma_src_bar; a.ldg = ld_src; a.self = 1;
        if (n_batch == 1) return hip_status(vpm::launch_backward(dtype, true, true, stretch, sym, a, st));
        return hip_status(backward_batched(dtype, n_batch, src_off, tgt_off, true, true, stretch, sym, a, false,
                                           workspace, st));
    }
    // Sources' gradients: lane = source (role B), loop = targets.
    a.xl = x_src; a.gl = gamma_src; a.sl = sigma_src; a.ubl = nullptr; a.sbl = nullptr;
    a.ldl = ld_src; a.nl = n_src;
    a.xo = x_tgt; a.go = gamma_tgt; a.so = sigma_tgt; a.ubo = u_bar; a.sbo = dgamma_bar;
    a.ldo = ld_tgt; a.no = n_tgt;
    a.xbar = x_src_bar; a.gbar = gamma_src_bar; a.ldg = ld_src; a.self = 0;
    hipError_t e = n_batch == 1 ? vpm::launch_backward(dtype, false, true, stretch, sym, a, st)
                                : backward_batched(dtype, n_batch, src_off, tgt_off, false, true, stretch, sym, a,
                                                   false, workspace, st);
    if (e != hipSuccess) return VPM_ERR_HIP;
    if (want_tgt) {
        // Targets' gradients: lane = target (role A), loop = sources.
        vpm::BwdArgs b;
        b.xl = x_tgt; b.gl = gamma_tgt; b.sl = sigma_tgt; b.ubl = u_bar; b.sbl = dgamma_bar;
        b.ldl = ld_tgt; b.nl = n_tgt;
        b.xo = x_src; b.go = gamma_src; b.so = sigma_src; b.ubo = nullptr; b.sbo = nullptr;
        b.ldo = ld_src; b.no = n_src;
        b.xbar = x_tgt_bar; b.gbar = gamma_tgt_bar; b.ldg = ld_tgt; b.self = 0;
        e = n_batch == 1 ? vpm::launch_backward(dtype, true, false, stretch, sym, b, st)
                         : backward_batched(dtype, n_batch, src_off, tgt_off, true, false, stretch, sym, b, true,
                                            workspace, st);
        if (e != hipSuccess) return VPM_ERR_HIP;
    }
    return VPM_OK;
}

size_t vpm_backward_workspace_size(int32_t dtype, int32_t n_batch, const int64_t* src_off, const int64_t* tgt_off) {
    if (!dtype_ok(dtype) || n_batch < 1 || check_offsets(n_batch, src_off) != VPM_OK) return 0;
    if (n_batch == 1) return 0;
    if (!tgt_off) tgt_off = src_off;
    if (check_offsets(n_batch, tgt_off) != VPM_OK) return 0;
    return backward_queue_layout(n_batch, src_off, tgt_off).total;
}

// State arrays may be FP64 while F and the evaluation copies are FP32 (mixed program);
// otherwise both types must match.
static bool stage_types_ok(int32_t dtype, int32_t state_dtype) {
    return dtype_ok(dtype) && dtype_ok(state_dtype) && (state_dtype == dtype || state_dtype == kDtypeF64);
}

vpm_status vpm_rk3_stage(int32_t dtype, int32_t state_dtype, int32_t stage, int64_t n, double dt, void* x,
                         void* gamma, void* qx, void* qg, const void* u, const void* dgamma, int64_t ld,
                         void* x_eval, void* gamma_eval, void* stream) {
    if (!stage_types_ok(dtype, state_dtype)) return VPM_ERR_DTYPE;
    if (stage < 0 || stage > 2) return VPM_ERR_ENUM;
    if (n < 0 || ld < n) return VPM_ERR_SIZE;
    if (!(dt == dt)) return VPM_ERR_SIZE;
    if (n > 0 && (!x || !gamma || !qx || !qg || !u || !dgamma)) return VPM_ERR_NULL;
    if ((x_eval == nullptr) != (gamma_eval == nullptr)) return VPM_ERR_NULL;
    const size_t es = elem_size(dtype), ss = elem_size(state_dtype);
    const Range rs[8] = {span(x, 3, ld, n, ss),  span(gamma, 3, ld, n, ss),  span(qx, 3, ld, n, ss),
                         span(qg, 3, ld, n, ss), span(u, 3, ld, n, es),      span(dgamma, 3, ld, n, es),
                         span(x_eval, 3, ld, n, es), span(gamma_eval, 3, ld, n, es)};
    for (int i = 0; i < 8; ++i)
        for (int j = i + 1; j < 8; ++j)
            if (overlap(rs[i], rs[j])) return VPM_ERR_ALIAS;
    if (n == 0) return VPM_OK;
    return hip_status(vpm::launch_rk3_stage(dtype, state_dtype, stage, n, dt, x, gamma, qx, qg, u, dgamma, ld,
                                            x_eval, gamma_eval, static_cast<hipStream_t>(stream)));
}

vpm_status vpm_rk3_stage_backward(int32_t dtype, int32_t state_dtype, int32_t stage, int64_t n, double dt,
                                  const void* x_bar, const void* gamma_bar, void* qx_bar, void* qg_bar,
                                  void* u_seed, void* dgamma_seed, int64_t ld, void* stream) {
    if (!stage_types_ok(dtype, state_dtype)) return VPM_ERR_DTYPE;
    if (stage < 0 || stage > 2) return VPM_ERR_ENUM;
    if (n < 0 || ld < n) return VPM_ERR_SIZE;
    if (!(dt == dt)) return VPM_ERR_SIZE;
    if (n > 0 && (!x_bar || !gamma_bar || !qx_bar || !qg_bar || !u_seed || !dgamma_seed)) return VPM_ERR_NULL;
    const size_t es = elem_size(dtype), ss = elem_size(state_dtype);
    const Range rs[6] = {span(x_bar, 3, ld, n, ss),  span(gamma_bar, 3, ld, n, ss),
                         span(qx_bar, 3, ld, n, ss), span(qg_bar, 3, ld, n, ss),
                         span(u_seed, 3, ld, n, es), span(dgamma_seed, 3, ld, n, es)};
    for (int i = 0; i < 6; ++i)
        for (int j = i + 1; j < 6; ++j)
            if (overlap(rs[i], rs[j])) return VPM_ERR_ALIAS;
    if (n == 0) return VPM_OK;
    return hip_status(vpm::launch_rk3_stage_bwd(dtype, state_dtype, stage, n, dt, x_bar, gamma_bar, qx_bar,
                                                qg_bar, u_seed, dgamma_seed, ld,
                                                static_cast<hipStream_t>(stream)));
}

vpm_status vpm_convert(int32_t src_dtype, int32_t dst_dtype, int64_t n, const void* src, int64_t ld_src, void* dst,
                       int64_t ld_dst, int32_t accumulate, void* stream) {
    if (!dtype_ok(src_dtype) || !dtype_ok(dst_dtype)) return VPM_ERR_DTYPE;
    if (n < 0 || ld_src < n || ld_dst < n) return VPM_ERR_SIZE;
    if (accumulate != 0 && accumulate != 1) return VPM_ERR_ENUM;
    if (n > 0 && (!src || !dst)) return VPM_ERR_NULL;
    if (overlap(span(src, 3, ld_src, n, elem_size(src_dtype)), span(dst, 3, ld_dst, n, elem_size(dst_dtype))))
        return VPM_ERR_ALIAS;
    if (n == 0) return VPM_OK;
    return hip_status(vpm::launch_convert(src_dtype, dst_dtype, n, src, ld_src, dst, ld_dst, accumulate,
                                          static_cast<hipStream_t>(stream)));
}

vpm_status vpm_axial_loss(int32_t dtype, int64_t m, const void* u, int64_t ld, double* loss, void* u_bar,
                          const double* loss_bar, void* stream) {
    if (!dtype_ok(dtype)) return VPM_ERR_DTYPE;
    if (m < 0 || ld < m) return VPM_ERR_SIZE;
    if (m > 0 && !u) return VPM_ERR_NULL;
    if (!loss && !u_bar) return VPM_ERR_NULL;
    const size_t es = elem_size(dtype);
    const Range ru = span(u, 3, ld, m, es), rb = span(u_bar, 3, ld, m, es);
    const Range rl = span(loss, 1, 1, 1, sizeof(double)), rlb = span(loss_bar, 1, 1, 1, sizeof(double));
    if (overlap(ru, rb) || overlap(ru, rl) || overlap(rb, rl) || overlap(rl, rlb) || overlap(rb, rlb))
        return VPM_ERR_ALIAS;
    return hip_status(vpm::launch_axial_loss(dtype, m, u, ld, loss, u_bar, loss_bar,
                                             static_cast<hipStream_t>(stream)));
}

size_t vpm_diagnostics_workspace_size(void) {
    return size_t(vpm::kDiagBlocks) * vpm::kDiagSlots * sizeof(double);
}

vpm_status vpm_validate_inputs(int32_t dtype, int64_t n, const void* x, const void* gamma, const void* sigma,
                               int64_t ld, double* out, void* workspace, size_t ws_bytes, void* stream) {
    if (!dtype_ok(dtype)) return VPM_ERR_DTYPE;
    if (n < 0 || ld < n) return VPM_ERR_SIZE;
    if (!out) return VPM_ERR_NULL;
    if (n > 0 && (!x || !gamma || !sigma)) return VPM_ERR_NULL;
    if (!workspace || ws_bytes < vpm_diagnostics_workspace_size()) return VPM_ERR_WORKSPACE;
    const Range ro = span(out, 1, 13, 13, sizeof(double));
    const Range rw = span(workspace, 1, vpm_diagnostics_workspace_size(), vpm_diagnostics_workspace_size(), 1);
    if (overlap(ro, rw)) return VPM_ERR_ALIAS;
    const size_t es = elem_size(dtype);
    const Range ins[3] = {span(x, 3, ld, n, es), span(gamma, 3, ld, n, es), span(sigma, 1, ld, n, es)};
    for (const Range& r : ins)
        if (overlap(ro, r) || overlap(rw, r)) return VPM_ERR_ALIAS;
    return hip_status(vpm::launch_validate(dtype, n, x, gamma, sigma, ld, out, static_cast<double*>(workspace),
                                           static_cast<hipStream_t>(stream)));
}

size_t vpm_check_inputs_workspace_size(void) { return vpm_diagnostics_workspace_size() + kAlign; }

vpm_status vpm_check_inputs(int32_t dtype, int64_t n, const void* x, const void* gamma, const void* sigma,
                            int64_t ld, void* workspace, size_t ws_bytes, void* stream) {
    if (!workspace || ws_bytes < vpm_check_inputs_workspace_size()) return VPM_ERR_WORKSPACE;
    const size_t dws = vpm_diagnostics_workspace_size();
    double* out = reinterpret_cast<double*>(static_cast<unsigned char*>(workspace) + dws);
    vpm_status s = vpm_validate_inputs(dtype, n, x, gamma, sigma, ld, out, workspace, dws, stream);
    if (s != VPM_OK || n == 0) return s;
    double host[2] = {0.0, 0.0};
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (hipMemcpyAsync(host, out, sizeof(host), hipMemcpyDeviceToHost, st) != hipSuccess) return VPM_ERR_HIP;
    if (hipStreamSynchronize(st) != hipSuccess) return VPM_ERR_HIP;
    return (host[0] != 0.0 || host[1] != 0.0) ? VPM_ERR_INPUT : VPM_OK;
}

vpm_status vpm_autotune(int32_t dtype, int32_t n_batch, const int64_t* src_off, const void* x, const void* gamma,
                        const void* sigma, int64_t ld, void* u_scratch, void* dgamma_scratch, void* workspace,
                        size_t ws_bytes, int32_t reps, int32_t* variant_out, float* ms_out, void* stream) {
    if (dtype != kDtypeF32C) return VPM_ERR_DTYPE;
    if (n_batch < 1 || reps < 1 || reps > 1000) return VPM_ERR_SIZE;
    if (!src_off) return VPM_ERR_NULL;
    vpm_status s = check_offsets(n_batch, src_off);
    if (s != VPM_OK) return s;
    const int64_t n = src_off[n_batch];
    if (n < 1) return VPM_ERR_SIZE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    vpm_options o = default_options();
    o.self = 1;
    // every shape once (validation, first-launch costs), then reps timed runs of each
    for (int v = 1; v <= vpm::kNumF32Variants; ++v) {
        o.variant = v;
        s = eval_impl(dtype, n_batch, src_off, nullptr, x, gamma, sigma, ld, nullptr, nullptr, nullptr, 0, nullptr,
                      u_scratch, dgamma_scratch, nullptr, ld, o, workspace, ws_bytes, stream);
        if (s != VPM_OK) return s;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return VPM_ERR_HIP;
    }
    float best_ms[vpm::kNumF32Variants];
    s = VPM_OK;
    for (int v = 1; v <= vpm::kNumF32Variants && s == VPM_OK; ++v) {
        o.variant = v;
        float best = -1.0f;
        for (int r = 0; r < reps && s == VPM_OK; ++r) {
            if (hipEventRecord(e0, st) != hipSuccess) { s = VPM_ERR_HIP; break; }
            s = eval_impl(dtype, n_batch, src_off, nullptr, x, gamma, sigma, ld, nullptr, nullptr, nullptr, 0,
                          nullptr, u_scratch, dgamma_scratch, nullptr, ld, o, workspace, ws_bytes, stream);
            if (s != VPM_OK) break;
            float ms = 0.0f;
            if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                s = VPM_ERR_HIP;
                break;
            }
            if (best < 0.0f || ms < best) best = ms;
        }
        best_ms[v - 1] = best;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s != VPM_OK) return s;
    int pick = 1;
    for (int v = 2; v <= vpm::kNumF32Variants; ++v)
        if (best_ms[v - 1] < best_ms[pick - 1]) pick = v;
    {
        std::lock_guard<std::mutex> lock(g_mutex);
        g_plan[n_batch > 1 ? 1 : 0][plan_bucket(n)] = pick;
    }
    if (variant_out) *variant_out = pick;
    if (ms_out)
        for (int v = 0; v < vpm::kNumF32Variants; ++v) ms_out[v] = best_ms[v];
    return VPM_OK;
}

vpm_status vpm_fma_chain(int64_t n_lanes, int32_t fmas_per_chain, int32_t form, float* out,
                         int64_t* fma_instructions, void* stream) {
    if (n_lanes < 1 || n_lanes > INT32_MAX || fmas_per_chain < 4 || fmas_per_chain % 4 != 0) return VPM_ERR_SIZE;
    if (form < 0 || form > 4) return VPM_ERR_ENUM;
    if (!out) return VPM_ERR_NULL;
    const int64_t waves = (n_lanes + 63) / 64;
    // wavefront FP32 FMA instructions, a 16x16x4 matrix step counting as 16 of them
    const int64_t per_step = form < 3 ? vpm::fma_chain_count() : (form == 3 ? 16 : 16 + vpm::fma_chain_count());
    if (fma_instructions) *fma_instructions = waves * per_step * fmas_per_chain;
    return hip_status(vpm::launch_fma_chain(n_lanes, fmas_per_chain, form, out, static_cast<hipStream_t>(stream)));
}

vpm_status vpm_diagnostics(int32_t dtype, int64_t n, const void* x, const void* gamma, const void* u,
                           const void* dgamma, int64_t ld, double* out, void* workspace,
                           size_t ws_bytes, void* stream) {
    if (!dtype_ok(dtype)) return VPM_ERR_DTYPE;
    if (n < 0 || ld < n) return VPM_ERR_SIZE;
    if (!out) return VPM_ERR_NULL;
    if (n > 0 && (!x || !gamma || !u || !dgamma)) return VPM_ERR_NULL;
    if (!workspace || ws_bytes < vpm_diagnostics_workspace_size()) return VPM_ERR_WORKSPACE;
    const Range ro = span(out, 1, 13, 13, sizeof(double));
    const Range rw = span(workspace, 1, vpm_diagnostics_workspace_size(), vpm_diagnostics_workspace_size(), 1);
    if (overlap(ro, rw)) return VPM_ERR_ALIAS;
    const size_t es = elem_size(dtype);
    const Range ins[4] = {span(x, 3, ld, n, es), span(gamma, 3, ld, n, es), span(u, 3, ld, n, es),
                          span(dgamma, 3, ld, n, es)};
    for (const Range& r : ins)
        if (overlap(ro, r) || overlap(rw, r)) return VPM_ERR_ALIAS;
    return hip_status(vpm::launch_diagnostics(dtype, n, x, gamma, u, dgamma, ld, out,
                                              static_cast<double*>(workspace),
                                              static_cast<hipStream_t>(stream)));
}

}  // extern "C"

// ------------------------------------------------------------------ blade solve and wake management
extern "C" {

vpm_status vpm_aic_assemble(int64_t n, const double* c00, const double* c01, const double* c11, const double* c10,
                            int64_t ld_ring, const double* colloc, const double* normal, int64_t ld_col,
                            double core_radius, int32_t vatistas_n, double* aic, int64_t ld_aic, void* stream) {
    if (n < 1 || n > 32768 || ld_ring < n || ld_col < n || ld_aic < n) return VPM_ERR_SIZE;
    if (!c00 || !c01 || !c11 || !c10 || !colloc || !normal || !aic) return VPM_ERR_NULL;
    if (!(core_radius >= 0.0) || core_radius > 1e30) return VPM_ERR_SIZE;
    if (vatistas_n < 1 || vatistas_n > 16) return VPM_ERR_ENUM;
    const Range ra = span(aic, 1, n * ld_aic, n * ld_aic, sizeof(double));
    const Range ins[6] = {span(c00, 3, ld_ring, n, 8), span(c01, 3, ld_ring, n, 8), span(c11, 3, ld_ring, n, 8),
                          span(c10, 3, ld_ring, n, 8), span(colloc, 3, ld_col, n, 8), span(normal, 3, ld_col, n, 8)};
    for (const Range& r : ins)
        if (overlap(ra, r)) return VPM_ERR_ALIAS;
    return hip_status(vpm::launch_aic(n, c00, c01, c11, c10, ld_ring, colloc, normal, ld_col, core_radius, vatistas_n,
                                      aic, ld_aic, static_cast<hipStream_t>(stream)));
}

vpm_status vpm_lu_factor(int64_t n, double* a, int64_t lda, int32_t* ipiv, int32_t* info, void* stream) {
    if (n < 1 || n > 32768 || lda < n) return VPM_ERR_SIZE;
    if (!a || !ipiv || !info) return VPM_ERR_NULL;
    const Range ra = span(a, 1, n * lda, n * lda, sizeof(double));
    if (overlap(ra, span(ipiv, 1, n, n, 4)) || overlap(ra, span(info, 1, 1, 1, 4)) ||
        overlap(span(ipiv, 1, n, n, 4), span(info, 1, 1, 1, 4)))
        return VPM_ERR_ALIAS;
    return hip_status(vpm::launch_lu_factor(n, a, lda, ipiv, info, static_cast<hipStream_t>(stream)));
}

vpm_status vpm_lu_solve(int64_t n, const double* lu, int64_t lda, const int32_t* ipiv, double* b, void* stream) {
    if (n < 1 || n > 32768 || lda < n) return VPM_ERR_SIZE;
    if (!lu || !ipiv || !b) return VPM_ERR_NULL;
    const Range rb = span(b, 1, n, n, sizeof(double));
    if (overlap(rb, span(lu, 1, n * lda, n * lda, sizeof(double))) || overlap(rb, span(ipiv, 1, n, n, 4)))
        return VPM_ERR_ALIAS;
    return hip_status(vpm::launch_lu_solve(n, lu, lda, ipiv, b, static_cast<hipStream_t>(stream)));
}

vpm_status vpm_wake_shed(int32_t dtype, int32_t n_blades, int32_t n_span, const void* gamma_blade,
                         const int32_t* te_index, void* gamma_te_prev, void* trailed_out, void* shed_out,
                         void* stream) {
    if (!dtype_ok(dtype)) return VPM_ERR_DTYPE;
    if (n_blades < 1 || n_span < 1 || int64_t(n_blades) * (2 * int64_t(n_span) + 1) > INT32_MAX) return VPM_ERR_SIZE;
    if (!gamma_blade || !te_index || !gamma_te_prev || !trailed_out || !shed_out) return VPM_ERR_NULL;
    const size_t es = elem_size(dtype);
    const int64_t ns = int64_t(n_blades) * n_span, nt = int64_t(n_blades) * (n_span + 1);
    const Range rt = span(trailed_out, 1, nt, nt, es), rs = span(shed_out, 1, ns, ns, es),
                rp = span(gamma_te_prev, 1, ns, ns, es), ri = span(te_index, 1, ns, ns, 4);
    if (overlap(rt, rs) || overlap(rt, rp) || overlap(rs, rp) || overlap(rt, ri) || overlap(rs, ri) ||
        overlap(rp, ri))
        return VPM_ERR_ALIAS;
    if (overlap(rt, span(gamma_blade, 1, 1, 1, es)) || overlap(rs, span(gamma_blade, 1, 1, 1, es)))
        return VPM_ERR_ALIAS;
    return hip_status(vpm::launch_wake_shed(dtype, n_blades, n_span, gamma_blade, te_index, gamma_te_prev,
                                            trailed_out, shed_out, static_cast<hipStream_t>(stream)));
}

size_t vpm_wake_convert_workspace_size(int64_t n_lines) {
    if (n_lines < 0 || n_lines > INT32_MAX) return 0;
    return vpm::conv_workspace(n_lines);
}

vpm_status vpm_wake_convert(int32_t dtype, int64_t n_lines, const void* a, const void* b, int64_t ld_line,
                            const void* dgamma, const int32_t* tip_index, int32_t n_tip, int32_t n_max,
                            double sigma, int64_t capacity, void* x_out, void* gamma_out, void* sigma_out,
                            int64_t ld_out, int64_t* count_out, void* workspace, size_t ws_bytes, void* stream) {
    if (!dtype_ok(dtype)) return VPM_ERR_DTYPE;
    if (n_lines < 0 || n_lines > INT32_MAX || ld_line < n_lines || capacity < 0 || ld_out < capacity)
        return VPM_ERR_SIZE;
    if (n_tip < 1 || n_max < 1 || n_max > 1 << 20) return VPM_ERR_SIZE;
    if (!(sigma > 0.0) || sigma > 1e30) return VPM_ERR_SIZE;
    if (!count_out) return VPM_ERR_NULL;
    if (n_lines > 0 && (!a || !b || !dgamma || !tip_index)) return VPM_ERR_NULL;
    if (capacity > 0 && (!x_out || !gamma_out || !sigma_out)) return VPM_ERR_NULL;
    const size_t need = vpm::conv_workspace(n_lines);
    if (!workspace || ws_bytes < need) return VPM_ERR_WORKSPACE;
    const size_t es = elem_size(dtype);
    const Range outs[4] = {span(x_out, 3, ld_out, capacity, es), span(gamma_out, 3, ld_out, capacity, es),
                           span(sigma_out, 1, ld_out, capacity, es), span(count_out, 1, 1, 1, 8)};
    const Range ins[5] = {span(a, 3, ld_line, n_lines, es), span(b, 3, ld_line, n_lines, es),
                          span(dgamma, 1, ld_line, n_lines, es), span(tip_index, 1, n_lines, n_lines, 4),
                          span(workspace, 1, int64_t(ws_bytes), int64_t(ws_bytes), 1)};
    for (int i = 0; i < 4; ++i) {
        for (const Range& r : ins)
            if (overlap(outs[i], r)) return VPM_ERR_ALIAS;
        for (int j = i + 1; j < 4; ++j)
            if (overlap(outs[i], outs[j])) return VPM_ERR_ALIAS;
    }
    for (int i = 0; i < 4; ++i)
        if (overlap(ins[4], ins[i])) return VPM_ERR_ALIAS;
    return hip_status(vpm::launch_wake_convert(dtype, n_lines, a, b, ld_line, dgamma, tip_index, n_tip, n_max, sigma,
                                               capacity, x_out, gamma_out, sigma_out, ld_out, count_out, workspace,
                                               static_cast<hipStream_t>(stream)));
}


vpm_status vpm_aic_update(int64_t n, const double* base, int64_t ld_base, double* out, int64_t ld_out,
                          const double* colloc, const double* normal, int64_t ld_col, int64_t m, const double* r00,
                          const double* r01, const double* r11, const double* r10, int64_t ld_ring,
                          const int32_t* ring_of_col, double core_radius, int32_t vatistas_n, void* stream) {
    if (n < 1 || n > 32768 || ld_base < n || ld_out < n || ld_col < n || m < 0 || ld_ring < m) return VPM_ERR_SIZE;
    if (!base || !out || !colloc || !normal || !ring_of_col) return VPM_ERR_NULL;
    if (m > 0 && (!r00 || !r01 || !r11 || !r10)) return VPM_ERR_NULL;
    if (!(core_radius >= 0.0) || core_radius > 1e30) return VPM_ERR_SIZE;
    if (vatistas_n < 1 || vatistas_n > 16) return VPM_ERR_ENUM;
    const Range ro = span(out, 1, n * ld_out, n * ld_out, 8), rb = span(base, 1, n * ld_base, n * ld_base, 8);
    if (overlap(ro, rb) && !(base == out && ld_base == ld_out)) return VPM_ERR_ALIAS;
    const Range ins[7] = {span(colloc, 3, ld_col, n, 8), span(normal, 3, ld_col, n, 8), span(r00, 3, ld_ring, m, 8),
                          span(r01, 3, ld_ring, m, 8),   span(r11, 3, ld_ring, m, 8),  span(r10, 3, ld_ring, m, 8),
                          span(ring_of_col, 1, n, n, 4)};
    for (const Range& r : ins)
        if (overlap(ro, r)) return VPM_ERR_ALIAS;
    return hip_status(vpm::launch_aic_update(n, base, ld_base, out, ld_out, colloc, normal, ld_col, m, r00, r01, r11,
                                             r10, ld_ring, ring_of_col, core_radius, vatistas_n,
                                             static_cast<hipStream_t>(stream)));
}

vpm_status vpm_neumann_rhs(int32_t dtype, int64_t n, const double* colloc, const double* normal, int64_t ld_col,
                           const void* u, int64_t ld_u, const double* v_inf, const double* omega, double* rhs,
                           void* stream) {
    if (!dtype_ok(dtype)) return VPM_ERR_DTYPE;
    if (n < 0 || ld_col < n || ld_u < n || n > INT32_MAX) return VPM_ERR_SIZE;
    if (!v_inf || !omega) return VPM_ERR_NULL;
    if (n == 0) return VPM_OK;
    if (!colloc || !normal || !u || !rhs) return VPM_ERR_NULL;
    const Range rr = span(rhs, 1, n, n, 8);
    if (overlap(rr, span(colloc, 3, ld_col, n, 8)) || overlap(rr, span(normal, 3, ld_col, n, 8)) ||
        overlap(rr, span(u, 3, ld_u, n, elem_size(dtype))))
        return VPM_ERR_ALIAS;
    return hip_status(vpm::launch_neumann_rhs(dtype, n, colloc, normal, ld_col, u, ld_u, v_inf, omega, rhs,
                                              static_cast<hipStream_t>(stream)));
}

vpm_status vpm_rk3_advect(int32_t dtype, int32_t stage, int64_t n, double dt, void* x, void* qx, const void* u,
                          void* gamma, void* qg, const void* dgamma, int64_t ld, const double* v_inf, void* stream) {
    if (!dtype_ok(dtype)) return VPM_ERR_DTYPE;
    if (stage < 0 || stage > 2) return VPM_ERR_ENUM;
    if (n < 0 || ld < n || n > INT32_MAX || !(dt == dt) || fabs(dt) > 1e30) return VPM_ERR_SIZE;
    if (!v_inf) return VPM_ERR_NULL;
    if (n == 0) return VPM_OK;
    if (!x || !qx || !u) return VPM_ERR_NULL;
    if ((gamma == nullptr) != (qg == nullptr) || (gamma && !dgamma)) return VPM_ERR_NULL;
    const size_t es = elem_size(dtype);
    const Range rs[6] = {span(x, 3, ld, n, es),     span(qx, 3, ld, n, es), span(gamma, 3, ld, n, es),
                         span(qg, 3, ld, n, es),    span(u, 3, ld, n, es),  span(gamma ? dgamma : nullptr, 3, ld, n, es)};
    for (int i = 0; i < 6; ++i)
        for (int j = i + 1; j < 6; ++j)
            if (overlap(rs[i], rs[j])) return VPM_ERR_ALIAS;
    return hip_status(vpm::launch_rk3_advect(dtype, stage, n, dt, x, qx, u, gamma, qg, dgamma, ld, v_inf,
                                             static_cast<hipStream_t>(stream)));
}

}  // extern "C"
