// kernels.h -- internal interface between the C-ABI layer and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

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
// chain), halo H run before each segment, checkpoint spacing CK.
struct SegPlan {
    int64_t L;
    int64_t H;
    int64_t CK;
};

// Process-wide tuning: target lanes per launch, shortest segment, halo.
struct SegTuning {
    int64_t target_lanes;
    int64_t min_segment;
    int64_t halo;
};
SegTuning &seg_tuning();
SegPlan seg_plan(int64_t num_chains, int64_t n);

template <typename T>
size_t chain_prox_ws_bytes(const ChainBatch &b, const SegPlan &plan);

template <typename T>
hipError_t launch_chain_prox(const ChainBatch &b, const T *y, const T *w, T w_scalar, T *x, void *workspace,
                             const SegPlan &plan, hipStream_t stream);

// Up to kMaxChainBatches uniform batches in one launch (see tv_chain_prox_multi).
constexpr int kMaxChainBatches = 8;
template <typename T>
hipError_t launch_chain_prox_multi(int nb, const ChainBatch *bs, const T *const *y, const T *const *w,
                                   const double *w_scalar, T *const *x, void *workspace, const SegPlan &plan,
                                   hipStream_t stream);

template <typename T>
hipError_t launch_chain_adjoint(const ChainBatch &b, const T *x, const T *g, T *gy, T *gw,
                                int w_per_edge, hipStream_t stream);

}  // namespace tvc
