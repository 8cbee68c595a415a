// api_chain.hip -- C ABI of the batched chain prox and its adjoint.
#include <math.h>

#include <map>
#include <mutex>

#include "../../include/tvchain.h"
#include "kernels.h"
#include "tv2d_common.h"

namespace tvc {

static const SegTuning kDefaultTuning{int64_t(1) << 17, 128, 128, kRingSlots};

SegTuning &seg_tuning() {
    static SegTuning t = kDefaultTuning;
    return t;
}

static int64_t round_tile(int64_t v) { return (v + kTile - 1) / kTile * kTile; }

// Enough segments per chain that the launch has about target_lanes lanes,
// with segments no shorter than min_segment; L, H and CK are tile multiples.
SegPlan seg_default_plan(int64_t num_chains, int64_t n) {
    const SegTuning &t = seg_tuning();
    SegPlan p;
    int64_t S = num_chains > 0 ? (t.target_lanes + num_chains - 1) / num_chains : 1;
    const int64_t smax = (n + t.min_segment - 1) / t.min_segment;
    if (S > smax) S = smax;
    if (S < 1) S = 1;
    p.L = round_tile((n + S - 1) / S);
    if (p.L < kTile) p.L = kTile;
    p.H = round_tile(t.halo);
    p.CK = 16;  // checkpoints at a + 16, 32, 64, 128 (tile multiples)
    p.K = (int)t.ring_slots;
    return p;
}

// Plans chosen by the autotuner, per (kind, chains, length).
namespace {
struct TunedKey {
    int kind;
    int64_t C, n;
    bool operator<(const TunedKey &o) const {
        return kind != o.kind ? kind < o.kind : (C != o.C ? C < o.C : n < o.n);
    }
};
std::mutex g_tuned_mu;
std::map<TunedKey, SegPlan> &tuned_map() {
    static std::map<TunedKey, SegPlan> m;
    return m;
}
}  // namespace

SegPlan seg_plan(int64_t num_chains, int64_t n, int kind) {
    {
        std::lock_guard<std::mutex> lk(g_tuned_mu);
        auto it = tuned_map().find(TunedKey{kind, num_chains, n});
        if (it != tuned_map().end()) return it->second;
    }
    return seg_default_plan(num_chains, n);
}

void seg_set_tuned(int kind, int64_t num_chains, int64_t n, const SegPlan &p) {
    std::lock_guard<std::mutex> lk(g_tuned_mu);
    tuned_map()[TunedKey{kind, num_chains, n}] = p;
}

void seg_clear_tuned() {
    std::lock_guard<std::mutex> lk(g_tuned_mu);
    tuned_map().clear();
}

// Host-side checks of a layout; no HIP call.
static bool layout_ok(const tv_chain_layout *L, tv_dtype dt) {
    if (!L) return false;
    if (dt != TV_F32 && dt != TV_F64) return false;
    if (L->num_chains < 0) return false;
    if (L->num_chains == 0) return true;
    if (L->length < 1) return false;
    const int64_t lim = (dt == TV_F32) ? (int64_t(1) << 24) : (int64_t(1) << 31) - 8;
    if (L->length >= lim) return false;
    if (!L->offsets) {
        if (L->elem_stride < 1) return false;
        if (L->num_chains > 1 && L->chain_stride < 1) return false;
    }
    return true;
}

static ChainBatch to_batch(const tv_chain_layout *L) {
    ChainBatch b;
    b.num_chains = L->num_chains;
    b.n = L->length;
    b.es = L->elem_stride;
    b.cs = L->chain_stride;
    b.offsets = L->offsets;
    return b;
}

// Byte range [lo, hi) touched by a uniform layout's elements starting at p
// (CSR layouts: only the base pointer is known on the host).
static void layout_span(const tv_chain_layout *L, tv_dtype dt, const void *p, uintptr_t *lo, uintptr_t *hi) {
    const size_t es = dt == TV_F32 ? 4 : 8;
    const uintptr_t b = (uintptr_t)p;
    *lo = b;
    if (L->offsets || L->num_chains < 1) {
        *hi = b + es;
        return;
    }
    const int64_t last = (L->num_chains - 1) * (L->num_chains > 1 ? L->chain_stride : 0) +
                         (L->length - 1) * L->elem_stride;
    *hi = b + (uintptr_t)(last + 1) * es;
}

// True if the output may overlap an input: segments of one chain run in
// parallel and re-read their input after neighbouring segments have written
// their output, so x must not share memory with y (or w).
static bool overlaps(const tv_chain_layout *Lx, const void *x, const tv_chain_layout *Ly, const void *y,
                     tv_dtype dt) {
    if (!x || !y) return false;
    if (x == y) return true;
    uintptr_t a0, a1, b0, b1;
    layout_span(Lx, dt, x, &a0, &a1);
    layout_span(Ly, dt, y, &b0, &b1);
    return a0 < b1 && b0 < a1;
}

// Room for any plan the autotuner may choose for this shape.
static size_t prox_ws_bytes(const tv_chain_layout *L, tv_dtype dt) {
    return dt == TV_F32 ? seg_bytes_max<float>(L->num_chains, L->length, kPlanChain)
                        : seg_bytes_max<double>(L->num_chains, L->length, kPlanChain);
}

static tv_status device_check() {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n < 1) return TV_ERR_NO_DEVICE;
    return TV_OK;
}

// Times one launch of the given plan (after one untimed run) with HIP events.
template <typename T>
hipError_t time_multi(int nb, const ChainBatch *bs, const void *const *y, const void *const *w,
                             const double *w_scalar, void *const *x, void *workspace, const SegPlan &plan,
                             hipStream_t stream, int reps, float *ms) {
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e != hipSuccess) return e;
    e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        hipEventDestroy(e0);
        return e;
    }
    auto run = [&]() {
        return launch_chain_prox_multi<T>(nb, bs, (const T *const *)y, (const T *const *)w, w_scalar,
                                          (T *const *)x, workspace, plan, stream);
    };
    e = run();
    if (e == hipSuccess) e = hipEventRecord(e0, stream);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = run();
    if (e == hipSuccess) e = hipEventRecord(e1, stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
    if (e == hipSuccess) *ms /= (float)reps;
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return e;
}

// Fixed device scratch of tv_chain_prox_noalloc: one copy per GPU the library
// runs on, held until the process ends.  Host code never passes the array's
// name to a kernel (on the host it is only a stand-in); it uses the device
// address obtained once per device with hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[TV_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];
}  // namespace

// The current device's scratch address (looked up on the first call per
// device, with that device current).
static tv_status scratch_address(void **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return TV_ERR_NO_DEVICE;
    if (dev >= kMaxDevices) return TV_ERR_NO_DEVICE;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return TV_ERR_HIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return TV_OK;
}

}  // namespace tvc

using namespace tvc;

extern "C" {

const char *tv_status_string(tv_status s) {
    static_assert(sizeof(tv_status) == sizeof(int) && sizeof(tv_dtype) == sizeof(int), "int-sized enums");
    switch (s) {
    case TV_OK: return "ok";
    case TV_ERR_INVALID_ARG: return "invalid argument";
    case TV_ERR_WORKSPACE: return "workspace missing or too small";
    case TV_ERR_NO_DEVICE: return "no HIP device";
    case TV_ERR_HIP: return "HIP runtime error";
    case TV_ERR_NOT_CONVERGED: return "duality gap tolerance not reached within max_iter";
    case TV_ERR_NONFINITE: return "non-finite duality gap";
    }
    return "unknown status";
}

size_t tv_chain_prox_workspace(const tv_chain_layout *layout, tv_dtype dtype) {
    if (!layout_ok(layout, dtype)) return 0;
    if (layout->num_chains == 0) return 0;
    return prox_ws_bytes(layout, dtype);
}

tv_status tv_chain_prox(const tv_chain_layout *layout, tv_dtype dtype, const void *y, const void *w,
                        double w_scalar, void *x, void *workspace, size_t workspace_bytes,
                        hipStream_t stream) {
    if (!layout_ok(layout, dtype)) return TV_ERR_INVALID_ARG;
    if (layout->num_chains == 0) return TV_OK;
    if (!y || !x) return TV_ERR_INVALID_ARG;
    if (!w && !(isfinite(w_scalar) && w_scalar >= 0.0)) return TV_ERR_INVALID_ARG;
    if (overlaps(layout, x, layout, y, dtype) || overlaps(layout, x, layout, w, dtype)) return TV_ERR_INVALID_ARG;
    const ChainBatch b = to_batch(layout);
    const SegPlan plan = seg_plan(b.num_chains, b.n);
    const size_t need = dtype == TV_F32 ? chain_prox_ws_bytes<float>(b, plan) : chain_prox_ws_bytes<double>(b, plan);
    if (!workspace || workspace_bytes < need) return TV_ERR_WORKSPACE;
    tv_status st = device_check();
    if (st != TV_OK) return st;
    hipError_t e;
    if (dtype == TV_F32)
        e = launch_chain_prox<float>(b, (const float *)y, (const float *)w, (float)w_scalar, (float *)x,
                                     workspace, plan, stream);
    else
        e = launch_chain_prox<double>(b, (const double *)y, (const double *)w, w_scalar, (double *)x,
                                      workspace, plan, stream);
    return e == hipSuccess ? TV_OK : TV_ERR_HIP;
}

tv_status tv_chain_prox_noalloc(const tv_chain_layout *layout, tv_dtype dtype, const void *y, const void *w,
                                double w_scalar, void *x, hipStream_t stream) {
    if (!layout_ok(layout, dtype)) return TV_ERR_INVALID_ARG;
    if (layout->num_chains == 0) return TV_OK;
    if (!y || !x) return TV_ERR_INVALID_ARG;
    if (!w && !(isfinite(w_scalar) && w_scalar >= 0.0)) return TV_ERR_INVALID_ARG;
    if (overlaps(layout, x, layout, y, dtype) || overlaps(layout, x, layout, w, dtype)) return TV_ERR_INVALID_ARG;
    const ChainBatch b = to_batch(layout);
    const SegPlan plan = seg_plan(b.num_chains, b.n);
    const size_t need = dtype == TV_F32 ? chain_prox_ws_bytes<float>(b, plan) : chain_prox_ws_bytes<double>(b, plan);
    if (need > TV_NOALLOC_SCRATCH_BYTES) return TV_ERR_WORKSPACE;
    tv_status st = device_check();
    if (st != TV_OK) return st;
    void *ws = nullptr;
    st = scratch_address(&ws);
    if (st != TV_OK) return st;
    hipError_t e;
    if (dtype == TV_F32)
        e = launch_chain_prox<float>(b, (const float *)y, (const float *)w, (float)w_scalar, (float *)x, ws, plan,
                                     stream);
    else
        e = launch_chain_prox<double>(b, (const double *)y, (const double *)w, w_scalar, (double *)x, ws, plan,
                                      stream);
    return e == hipSuccess ? TV_OK : TV_ERR_HIP;
}

// ---- general unaries and asymmetric weights ----

static size_t dp_ws_bytes(const tv_chain_layout *L, tv_dtype dt) {
    const int64_t C = L->num_chains, n = L->length;
    return dt == TV_F32 ? chain_dp_ws_bytes<float>(C, n, seg_bytes_max<float, double>(C, n, kPlanDp))
                        : chain_dp_ws_bytes<double>(C, n, seg_bytes_max<double, double>(C, n, kPlanDp));
}

static size_t dp_ws_bytes_plan(const tv_chain_layout *L, tv_dtype dt, const SegPlan &p) {
    const int64_t C = L->num_chains, n = L->length;
    return dt == TV_F32 ? chain_dp_ws_bytes<float>(C, n, seg_ws_bytes_plan<float, double>(C, n, p))
                        : chain_dp_ws_bytes<double>(C, n, seg_ws_bytes_plan<double, double>(C, n, p));
}

static tv_status dp_args(const tv_chain_layout *L, tv_dtype dt, const void *a, const void *b, const void *wm,
                         const void *wp, void *x) {
    if (!layout_ok(L, dt)) return TV_ERR_INVALID_ARG;
    if (L->num_chains == 0) return TV_OK;
    if (!b || !wm || !wp || !x) return TV_ERR_INVALID_ARG;
    if (overlaps(L, x, L, a, dt) || overlaps(L, x, L, b, dt) || overlaps(L, x, L, wm, dt) ||
        overlaps(L, x, L, wp, dt))
        return TV_ERR_INVALID_ARG;
    return TV_OK;
}

static hipError_t dp_launch(const tv_chain_layout *L, tv_dtype dt, const void *a, const void *b, const void *wm,
                            const void *wp, void *x, void *ws, const SegPlan &plan, hipStream_t st) {
    const ChainBatch bt = to_batch(L);
    if (dt == TV_F32)
        return launch_chain_dp<float>(bt, (const float *)a, (const float *)b, (const float *)wm, (const float *)wp,
                                      (float *)x, ws, plan, st);
    return launch_chain_dp<double>(bt, (const double *)a, (const double *)b, (const double *)wm,
                                   (const double *)wp, (double *)x, ws, plan, st);
}

size_t tv_chain_dp_workspace(const tv_chain_layout *layout, tv_dtype dtype) {
    if (!layout_ok(layout, dtype) || layout->num_chains == 0) return 0;
    return dp_ws_bytes(layout, dtype);
}

tv_status tv_chain_dp(const tv_chain_layout *layout, tv_dtype dtype, const void *a, const void *b, const void *wm,
                      const void *wp, void *x, void *workspace, size_t workspace_bytes, hipStream_t stream) {
    tv_status st = dp_args(layout, dtype, a, b, wm, wp, x);
    if (st != TV_OK || layout->num_chains == 0) return st;
    const SegPlan plan = seg_plan(layout->num_chains, layout->length, kPlanDp);
    if (!workspace || workspace_bytes < dp_ws_bytes_plan(layout, dtype, plan)) return TV_ERR_WORKSPACE;
    st = device_check();
    if (st != TV_OK) return st;
    return dp_launch(layout, dtype, a, b, wm, wp, x, workspace, plan, stream) == hipSuccess ? TV_OK : TV_ERR_HIP;
}

tv_status tv_chain_dp_autotune(const tv_chain_layout *layout, tv_dtype dtype, const void *a, const void *b,
                               const void *wm, const void *wp, void *x, void *workspace, size_t workspace_bytes,
                               hipStream_t stream, tv_tuning_result *chosen) {
    tv_status st = dp_args(layout, dtype, a, b, wm, wp, x);
    if (st != TV_OK || layout->num_chains == 0) return st;
    if (!workspace) return TV_ERR_WORKSPACE;
    st = device_check();
    if (st != TV_OK) return st;
    const int64_t C = layout->num_chains, n = layout->length;
    SegPlan cand[64];
    const int m = dtype == TV_F32 ? seg_candidates<float, double>(C, n, cand, 64)
                                  : seg_candidates<double, double>(C, n, cand, 64);
    int best = -1, tried = 0;
    float best_ms = 0.0f;
    for (int j = 0; j < m; ++j) {
        if (dp_ws_bytes_plan(layout, dtype, cand[j]) > workspace_bytes) continue;
        float ms = 0.0f;
        if (time_calls([&]() { return dp_launch(layout, dtype, a, b, wm, wp, x, workspace, cand[j], stream); },
                       stream, 3, &ms) != hipSuccess)
            return TV_ERR_HIP;
        ++tried;
        if (best < 0 || ms < best_ms) {
            best = j;
            best_ms = ms;
        }
    }
    if (best < 0) return TV_ERR_WORKSPACE;
    seg_set_tuned(kPlanDp, C, n, cand[best]);
    if (chosen) {
        chosen->segment_length = cand[best].L;
        chosen->halo = cand[best].H;
        chosen->ring_slots = cand[best].K;
        chosen->candidates = tried;
        chosen->ms = best_ms;
    }
    return TV_OK;
}

// ---- TV-l1 chain prox ----

size_t tv_chain_prox_l1_workspace(const tv_chain_layout *layout, tv_dtype dtype) {
    if (!layout_ok(layout, dtype) || layout->num_chains == 0) return 0;
    return dtype == TV_F32 ? chain_l1_ws_bytes<float>(layout->num_chains, layout->length)
                           : chain_l1_ws_bytes<double>(layout->num_chains, layout->length);
}

tv_status tv_chain_prox_l1(const tv_chain_layout *layout, tv_dtype dtype, const void *y, const void *d,
                           const void *w, double w_scalar, const void *c, double c_scalar, void *x,
                           void *workspace, size_t workspace_bytes, hipStream_t stream) {
    if (!layout_ok(layout, dtype)) return TV_ERR_INVALID_ARG;
    if (layout->num_chains == 0) return TV_OK;
    if (!y || !d || !x) return TV_ERR_INVALID_ARG;
    if (!w && !(isfinite(w_scalar) && w_scalar >= 0.0)) return TV_ERR_INVALID_ARG;
    if (!c && !(isfinite(c_scalar) && c_scalar >= 0.0)) return TV_ERR_INVALID_ARG;
    if (overlaps(layout, x, layout, y, dtype) || overlaps(layout, x, layout, d, dtype) ||
        overlaps(layout, x, layout, w, dtype) || overlaps(layout, x, layout, c, dtype))
        return TV_ERR_INVALID_ARG;
    if (!workspace || workspace_bytes < tv_chain_prox_l1_workspace(layout, dtype)) return TV_ERR_WORKSPACE;
    tv_status st = device_check();
    if (st != TV_OK) return st;
    const ChainBatch b = to_batch(layout);
    hipError_t e;
    if (dtype == TV_F32)
        e = launch_chain_l1<float>(b, (const float *)y, (const float *)d, (const float *)w, (float)w_scalar,
                                   (const float *)c, (float)c_scalar, (float *)x, workspace, stream);
    else
        e = launch_chain_l1<double>(b, (const double *)y, (const double *)d, (const double *)w, w_scalar,
                                    (const double *)c, c_scalar, (double *)x, workspace, stream);
    return e == hipSuccess ? TV_OK : TV_ERR_HIP;
}

tv_status tv_chain_prox_l1_autotune(const tv_chain_layout *layout, tv_dtype dtype, const void *y, const void *d,
                                    const void *w, double w_scalar, const void *c, double c_scalar, void *x,
                                    void *workspace, size_t workspace_bytes, hipStream_t stream,
                                    tv_tuning_result *chosen) {
    // argument checks and one launch with the current plan
    tv_status st = tv_chain_prox_l1(layout, dtype, y, d, w, w_scalar, c, c_scalar, x, workspace, workspace_bytes,
                                    stream);
    if (st != TV_OK || layout->num_chains == 0) return st;
    const int64_t C = layout->num_chains, n = layout->length;
    const ChainBatch b = to_batch(layout);
    SegPlan cand[64];
    // the TV-l1 set is FP64 for either data precision
    const int m = seg_candidates<double, TagJ<double>>(C, n, cand, 64);
    int best = -1, tried = 0;
    float best_ms = 0.0f;
    for (int j = 0; j < m; ++j) {
        const size_t need = seg_ws_bytes_plan<double, TagJ<double>>(C, n, cand[j]);
        if (need > workspace_bytes) continue;
        seg_set_tuned(kPlanL1, C, n, cand[j]);
        auto run = [&]() {
            return dtype == TV_F32
                       ? launch_chain_l1<float>(b, (const float *)y, (const float *)d, (const float *)w,
                                                (float)w_scalar, (const float *)c, (float)c_scalar, (float *)x,
                                                workspace, stream)
                       : launch_chain_l1<double>(b, (const double *)y, (const double *)d, (const double *)w, w_scalar,
                                                 (const double *)c, c_scalar, (double *)x, workspace, stream);
        };
        float ms = 0.0f;
        if (time_calls(run, stream, 3, &ms) != hipSuccess) return TV_ERR_HIP;
        ++tried;
        if (best < 0 || ms < best_ms) {
            best = j;
            best_ms = ms;
        }
    }
    if (best < 0) return TV_ERR_WORKSPACE;
    seg_set_tuned(kPlanL1, C, n, cand[best]);
    // x from the chosen plan (every plan gives the same bits)
    st = tv_chain_prox_l1(layout, dtype, y, d, w, w_scalar, c, c_scalar, x, workspace, workspace_bytes, stream);
    if (st != TV_OK) return st;
    if (hipStreamSynchronize(stream) != hipSuccess) return TV_ERR_HIP;
    if (chosen) {
        chosen->segment_length = cand[best].L;
        chosen->halo = cand[best].H;
        chosen->ring_slots = cand[best].K;
        chosen->candidates = tried;
        chosen->ms = best_ms;
    }
    return TV_OK;
}

// ---- trees ----

size_t tv_tree_dp_workspace(int64_t num_trees, int64_t num_nodes) {
    if (num_trees < 1 || num_nodes < 1) return 0;
    return tree_dp_ws_bytes(num_trees, num_nodes);
}

tv_status tv_tree_dp(tv_dtype dtype, int64_t num_trees, int64_t num_nodes, const int64_t *offsets,
                     const int64_t *parent, const void *a, const void *b, const void *c, const void *d,
                     const void *wm, const void *wp, void *x, void *workspace, size_t workspace_bytes,
                     hipStream_t stream) {
    if (dtype != TV_F32 && dtype != TV_F64) return TV_ERR_INVALID_ARG;
    if (num_trees < 0 || num_nodes < 0) return TV_ERR_INVALID_ARG;
    if (num_trees == 0 || num_nodes == 0) return TV_OK;
    if (!offsets || !parent || !b || !wm || !wp || !x || (c && !d)) return TV_ERR_INVALID_ARG;
    if (x == a || x == b || x == c || x == d || x == wm || x == wp) return TV_ERR_INVALID_ARG;
    if (!workspace || workspace_bytes < tv_tree_dp_workspace(num_trees, num_nodes)) return TV_ERR_WORKSPACE;
    tv_status st = device_check();
    if (st != TV_OK) return st;
    int bad = 0;
    hipError_t e;
    if (dtype == TV_F32)
        e = launch_tree_dp<float>(num_trees, num_nodes, offsets, parent, (const float *)a, (const float *)b,
                                  (const float *)c, (const float *)d, (const float *)wm, (const float *)wp,
                                  (float *)x, workspace, &bad, stream);
    else
        e = launch_tree_dp<double>(num_trees, num_nodes, offsets, parent, (const double *)a, (const double *)b,
                                   (const double *)c, (const double *)d, (const double *)wm, (const double *)wp,
                                   (double *)x, workspace, &bad, stream);
    if (e != hipSuccess) return TV_ERR_HIP;
    return bad ? TV_ERR_INVALID_ARG : TV_OK;
}

static_assert(kMaxChainBatches == TV_MAX_CHAIN_BATCHES, "batch limit of the ABI");

static bool multi_ok(int nb, const tv_chain_layout *layouts, tv_dtype dtype, int64_t *C, int64_t *n) {
    if (nb < 1 || nb > kMaxChainBatches || !layouts) return false;
    *C = 0;
    *n = 0;
    for (int b = 0; b < nb; ++b) {
        if (!layout_ok(&layouts[b], dtype) || layouts[b].offsets) return false;
        *C += layouts[b].num_chains;
        if (layouts[b].num_chains > 0 && layouts[b].length > *n) *n = layouts[b].length;
    }
    return true;
}

size_t tv_chain_prox_multi_workspace(int num_batches, const tv_chain_layout *layouts, tv_dtype dtype) {
    int64_t C, n;
    if (!multi_ok(num_batches, layouts, dtype, &C, &n) || C == 0) return 0;
    return dtype == TV_F32 ? seg_bytes_max<float>(C, n, kPlanChain) : seg_bytes_max<double>(C, n, kPlanChain);
}

tv_status tv_chain_prox_multi(int num_batches, const tv_chain_layout *layouts, tv_dtype dtype,
                              const void *const *y, const void *const *w, const double *w_scalar,
                              void *const *x, void *workspace, size_t workspace_bytes, hipStream_t stream) {
    int64_t C, n;
    if (!multi_ok(num_batches, layouts, dtype, &C, &n)) return TV_ERR_INVALID_ARG;
    if (C == 0) return TV_OK;
    if (!y || !x || (!w && !w_scalar)) return TV_ERR_INVALID_ARG;
    ChainBatch bs[kMaxChainBatches];
    for (int b = 0; b < num_batches; ++b) {
        if (layouts[b].num_chains > 0 && (!y[b] || !x[b] || (w && !w[b]))) return TV_ERR_INVALID_ARG;
        if (!w && !(isfinite(w_scalar[b]) && w_scalar[b] >= 0.0)) return TV_ERR_INVALID_ARG;
        for (int o = 0; o < num_batches; ++o) {
            if (overlaps(&layouts[b], x[b], &layouts[o], y[o], dtype)) return TV_ERR_INVALID_ARG;
            if (w && overlaps(&layouts[b], x[b], &layouts[o], w[o], dtype)) return TV_ERR_INVALID_ARG;
            if (o != b && overlaps(&layouts[b], x[b], &layouts[o], x[o], dtype)) return TV_ERR_INVALID_ARG;
        }
        bs[b] = to_batch(&layouts[b]);
    }
    const SegPlan plan = seg_plan(C, n);
    ChainBatch all{C, n, 1, n, nullptr};
    const size_t need = dtype == TV_F32 ? chain_prox_ws_bytes<float>(all, plan) : chain_prox_ws_bytes<double>(all, plan);
    if (!workspace || workspace_bytes < need) return TV_ERR_WORKSPACE;
    tv_status st = device_check();
    if (st != TV_OK) return st;
    hipError_t e;
    if (dtype == TV_F32)
        e = launch_chain_prox_multi<float>(num_batches, bs, (const float *const *)y, (const float *const *)w,
                                           w_scalar, (float *const *)x, workspace, plan, stream);
    else
        e = launch_chain_prox_multi<double>(num_batches, bs, (const double *const *)y, (const double *const *)w,
                                            w_scalar, (double *const *)x, workspace, plan, stream);
    return e == hipSuccess ? TV_OK : TV_ERR_HIP;
}

tv_status tv_chain_prox_autotune(int num_batches, const tv_chain_layout *layouts, tv_dtype dtype,
                                 const void *const *y, const void *const *w, const double *w_scalar,
                                 void *const *x, void *workspace, size_t workspace_bytes, hipStream_t stream,
                                 tv_tuning_result *chosen) {
    int64_t C, n;
    if (!multi_ok(num_batches, layouts, dtype, &C, &n)) return TV_ERR_INVALID_ARG;
    if (C == 0) return TV_OK;
    if (!y || !x || (!w && !w_scalar)) return TV_ERR_INVALID_ARG;
    ChainBatch bs[kMaxChainBatches];
    for (int b = 0; b < num_batches; ++b) {
        if (layouts[b].num_chains > 0 && (!y[b] || !x[b] || (w && !w[b]))) return TV_ERR_INVALID_ARG;
        if (!w && !(isfinite(w_scalar[b]) && w_scalar[b] >= 0.0)) return TV_ERR_INVALID_ARG;
        for (int o = 0; o < num_batches; ++o) {
            if (overlaps(&layouts[b], x[b], &layouts[o], y[o], dtype)) return TV_ERR_INVALID_ARG;
            if (w && overlaps(&layouts[b], x[b], &layouts[o], w[o], dtype)) return TV_ERR_INVALID_ARG;
            if (o != b && overlaps(&layouts[b], x[b], &layouts[o], x[o], dtype)) return TV_ERR_INVALID_ARG;
        }
        bs[b] = to_batch(&layouts[b]);
    }
    if (!workspace) return TV_ERR_WORKSPACE;
    tv_status st = device_check();
    if (st != TV_OK) return st;
    SegPlan cand[64];
    const int m = dtype == TV_F32 ? seg_candidates<float>(C, n, cand, 64) : seg_candidates<double>(C, n, cand, 64);
    int best = -1, tried = 0;
    float best_ms = 0.0f;
    for (int j = 0; j < m; ++j) {
        const size_t need = dtype == TV_F32 ? seg_ws_bytes_plan<float>(C, n, cand[j])
                                            : seg_ws_bytes_plan<double>(C, n, cand[j]);
        if (need > workspace_bytes) continue;
        float ms = 0.0f;
        const hipError_t e =
            dtype == TV_F32
                ? time_multi<float>(num_batches, bs, y, w, w_scalar, x, workspace, cand[j], stream, 3, &ms)
                : time_multi<double>(num_batches, bs, y, w, w_scalar, x, workspace, cand[j], stream, 3, &ms);
        if (e != hipSuccess) return TV_ERR_HIP;
        ++tried;
        if (best < 0 || ms < best_ms) {
            best = j;
            best_ms = ms;
        }
    }
    if (best < 0) return TV_ERR_WORKSPACE;
    seg_set_tuned(kPlanChain, C, n, cand[best]);
    if (chosen) {
        chosen->segment_length = cand[best].L;
        chosen->halo = cand[best].H;
        chosen->ring_slots = cand[best].K;
        chosen->candidates = tried;
        chosen->ms = best_ms;
    }
    return TV_OK;
}

void tv_autotune_clear(void) { seg_clear_tuned(); }

tv_status tv_set_tuning(const tv_tuning *t) {
    if (!t) {
        seg_tuning() = kDefaultTuning;
        return TV_OK;
    }
    if (t->target_lanes < 1 || t->min_segment < 1 || t->halo < 0) return TV_ERR_INVALID_ARG;
    if (t->ring_slots != 16 && t->ring_slots != 32 && t->ring_slots != 64 && t->ring_slots != 128)
        return TV_ERR_INVALID_ARG;
    seg_tuning() = SegTuning{t->target_lanes, t->min_segment, t->halo, t->ring_slots};
    return TV_OK;
}

tv_status tv_get_tuning(tv_tuning *t) {
    if (!t) return TV_ERR_INVALID_ARG;
    t->target_lanes = seg_tuning().target_lanes;
    t->min_segment = seg_tuning().min_segment;
    t->halo = seg_tuning().halo;
    t->ring_slots = seg_tuning().ring_slots;
    return TV_OK;
}

int64_t tv_chain_prox_segment_length(const tv_chain_layout *layout) {
    if (!layout || layout->num_chains < 1 || layout->length < 1) return 0;
    return seg_plan(layout->num_chains, layout->length).L;
}

size_t tv_chain_prox_backward_workspace(const tv_chain_layout *layout, tv_dtype dtype) {
    (void)layout;
    (void)dtype;
    return 0;
}

tv_status tv_chain_prox_backward(const tv_chain_layout *layout, tv_dtype dtype, const void *x,
                                 const void *grad_x, void *grad_y, void *grad_w, int w_per_edge,
                                 void *workspace, size_t workspace_bytes, hipStream_t stream) {
    (void)workspace;
    (void)workspace_bytes;
    if (!layout_ok(layout, dtype)) return TV_ERR_INVALID_ARG;
    if (layout->num_chains == 0) return TV_OK;
    if (!x || !grad_x) return TV_ERR_INVALID_ARG;
    if (!grad_y && !grad_w) return TV_OK;
    tv_status st = device_check();
    if (st != TV_OK) return st;
    const ChainBatch b = to_batch(layout);
    hipError_t e;
    if (dtype == TV_F32)
        e = launch_chain_adjoint<float>(b, (const float *)x, (const float *)grad_x, (float *)grad_y,
                                        (float *)grad_w, w_per_edge, stream);
    else
        e = launch_chain_adjoint<double>(b, (const double *)x, (const double *)grad_x, (double *)grad_y,
                                         (double *)grad_w, w_per_edge, stream);
    return e == hipSuccess ? TV_OK : TV_ERR_HIP;
}

}  // extern "C"
