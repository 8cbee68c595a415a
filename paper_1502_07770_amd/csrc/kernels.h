// kernels.h -- internal interface between the C-ABI layer and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

// A source that instantiates many kernel templates is compiled several times
// by the build, once per part (TVC_PART = 1 .. n), each part instantiating
// one subset; TVC_PART = 0 (the default, a single compilation) instantiates
// everything.
#ifndef TVC_PART
#define TVC_PART 0
#endif
#define TVC_IN_PART(k) (TVC_PART == 0 || TVC_PART == (k))

namespace tvc {

// Breakpoint slots of the per-lane LDS ring.  The deepest deque seen on the
// piecewise-constant / shapes workloads is ~15 breakpoints; chains that go
// deeper are solved with their deque in HBM.
#ifndef TVC_RING_SLOTS
#define TVC_RING_SLOTS 16
#endif
constexpr int kRingSlots = TVC_RING_SLOTS;
// Nodes per register tile: loads run this many nodes ahead of their use.
constexpr int kTile = 8;

struct ChainBatch {
    int64_t num_chains;
    int64_t n;               // uniform length (maximum length with offsets)
    int64_t es, cs;          // element / chain strides (uniform batches)
    const int64_t *offsets;  // CSR starts (device) or nullptr
};

// Segmentation of a launch: segment length L (S = ceil(n / L) segments per
// chain), halo H run before each segment, checkpoint spacing CK, and the
// number K of breakpoint slots of the LDS ring (16, 32; 64 or 128 for 8-byte entries).
struct SegPlan {
    int64_t L;
    int64_t H;
    int64_t CK;
    int K;
};

// Which launch a plan is for: the best segmentation depends on the problem's
// data source, so tuned plans are cached per kind and shape.
enum PlanKind {
    kPlanChain = 0,
    kPlan2dCol = 1,
    kPlan2dRow = 2,
    kPlanBatchCol = 3,
    kPlanBatchRow = 4,
    kPlanDp = 5,
    kPlanL1 = 6,
    kPlan2dRowL1 = 7,
    kPlan2dColL1 = 8,  // the TV-l1 solve's column (ROF dual) launch: deeper deques than ROF's
    kPlanKinds = 9
};

// Process-wide tuning: target lanes per launch, shortest segment, halo.
struct SegTuning {
    int64_t target_lanes;
    int64_t min_segment;
    int64_t halo;
    int64_t ring_slots;
};
SegTuning &seg_tuning();
// The plan used for a launch of num_chains chains of length <= n: the tuned
// plan of this kind and shape if one was chosen (tv_*_autotune), else the
// process-wide tuning.
SegPlan seg_plan(int64_t num_chains, int64_t n, int kind = kPlanChain);
SegPlan seg_default_plan(int64_t num_chains, int64_t n);
void seg_set_tuned(int kind, int64_t num_chains, int64_t n, const SegPlan &p);
void seg_clear_tuned();
// Tag of a TV-l1 breakpoint (slope tag and jump; defined in l1_core.h).
template <typename T> struct TagJ;

// Candidate plans for the autotuner (the default plan first); every workspace
// query reserves room for the largest of them, so a tuned plan always fits.
// G is the tag type of the deque entries (T when a_i = 1, FP64 otherwise).
template <typename T, typename G = T>
int seg_candidates(int64_t num_chains, int64_t n, SegPlan *out, int max_out);
template <typename T, typename G = T>
size_t seg_bytes_max(int64_t num_chains, int64_t n, int kind);

template <typename T>
size_t chain_prox_ws_bytes(const ChainBatch &b, const SegPlan &plan);
// Workspace bytes of one launch of num_chains chains of length <= n under plan.
template <typename T, typename G = T>
size_t seg_ws_bytes_plan(int64_t num_chains, int64_t n, const SegPlan &plan);

template <typename T>
hipError_t launch_chain_prox(const ChainBatch &b, const T *y, const T *w, T w_scalar, T *x, void *workspace,
                             const SegPlan &plan, hipStream_t stream);

// Up to kMaxChainBatches uniform batches in one launch (see tv_chain_prox_multi).
constexpr int kMaxChainBatches = 8;
template <typename T>
hipError_t launch_chain_prox_multi(int nb, const ChainBatch *bs, const T *const *y, const T *const *w,
                                   const double *w_scalar, T *const *x, void *workspace, const SegPlan &plan,
                                   hipStream_t stream);

// General unaries and asymmetric weights (see tv_chain_dp): workspace bytes
// with seg_bytes for the segmented kernels, and the launch.
template <typename T>
size_t chain_dp_ws_bytes(int64_t num_chains, int64_t n, size_t seg_bytes);
template <typename T>
hipError_t launch_chain_dp(const ChainBatch &b, const T *a, const T *bv, const T *wm, const T *wp, T *x,
                           void *workspace, const SegPlan &plan, hipStream_t stream);

// TV-l1 chain prox (see tv_chain_prox_l1): workspace bytes and the launch.
template <typename T>
size_t chain_l1_ws_bytes(int64_t num_chains, int64_t n);
template <typename T>
hipError_t launch_chain_l1(const ChainBatch &b, const T *y, const T *d, const T *w, T w_scalar, const T *c,
                           T c_scalar, T *x, void *workspace, hipStream_t stream);

// Algorithm 2 on a batch of trees (see tv_tree_dp); the launch reads the
// post-order check back into *bad_host and synchronizes the stream.
size_t tree_dp_ws_bytes(int64_t num_trees, int64_t num_nodes);
template <typename T>
hipError_t launch_tree_dp(int64_t num_trees, int64_t num_nodes, const int64_t *offsets, const int64_t *parent,
                          const T *a, const T *b, const T *c, const T *d, const T *wm, const T *wp, T *x,
                          void *workspace, int *bad_host, hipStream_t stream);

template <typename T>
hipError_t launch_chain_adjoint(const ChainBatch &b, const T *x, const T *g, T *gy, T *gw,
                                int w_per_edge, hipStream_t stream);

}  // namespace tvc
