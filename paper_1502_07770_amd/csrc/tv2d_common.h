// tv2d_common.h -- pieces shared by the single-image and batched 2D solvers.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "../../include/tvchain.h"
#include "kernels.h"

namespace tvc {

// Threads per block of the gap reductions (four wave64 rows per block).
constexpr int kGapBlock = 256;
// Rows per block of the column prefix sums of the gap.  The single-image and
// batched solvers sum in the same order (within a block from zero, blocks
// added left to right), so their gaps agree bit for bit.
constexpr int kGapRows = 64;

// Per-iteration scalars of the accelerated schedule, computed on the host in
// FP64 and read by the kernels from device memory, so that a chunk of
// iterations can be captured once in a HIP graph and replayed.
struct IterSched {
    double tau;     // tau_k
    double sigma;   // 1 / tau_k
    double theta;   // 1 / sqrt(1 + 2 tau_k)
    double inv1p;   // 1 / (1 + tau_k)
    double pscale;  // (1 + tau_k) / tau_k
    int64_t iter_after;  // k + 1
};
// Iterations whose schedule one upload holds (and the longest captured chunk).
constexpr int kSchedCap = 64;
// Iterations the autotuners run before timing candidate plans (even, so the
// state is back in the buffers of parity 0).  The chains' deques deepen as the
// dual variable builds up: timed after 8 iterations, the plans of a 4096^2
// ROF solve used 16-slot rings that later iterations outgrew (the overflowed
// chains then run sequentially), 3x slower to a gap of 1e-6 than 32 slots.
constexpr int kTuneWarm = 32;

__host__ __device__ __forceinline__ IterSched make_sched(double tau, int64_t k) {
    IterSched s;
    s.tau = tau;
    s.sigma = 1.0 / tau;
    s.theta = 1.0 / sqrt(1.0 + 2.0 * tau);
    s.inv1p = 1.0 / (1.0 + tau);
    s.pscale = (1.0 + tau) / tau;
    s.iter_after = k + 1;
    return s;
}

// Device-resident control of a 2D solve.  The host enqueues iterations
// without waiting on the device (up to max_iter, or a bounded lookahead of gap
// evaluations, see Lookahead below); the schedule is generated on the device,
// and once the stopping test passes (or the gap is not finite) `stop` is set
// and every later kernel of the solve returns at once.
struct SolveCtl {
    double tau;        // tau of the next iteration to schedule
    int64_t knext;     // index of the next iteration to schedule
    int32_t stop;      // 1: stopped; later launches do nothing
    int32_t status;    // the solve's status once stopped (TV_OK or TV_ERR_NONFINITE)
    int32_t n_active;  // batched solves: images still iterating
    uint32_t seq;      // the call's number, written to *host_stop at the stop
    uint64_t t0, t1;   // device wall clock at the first scheduled iteration and at the stop
    uint32_t *host_stop;  // pinned host word that mirrors the stop for the host (or null)
};

static __global__ void k_ctl_init(SolveCtl *c, double tau0, int n_active, uint32_t *host_stop, uint32_t seq) {
    if (threadIdx.x != 0) return;
    c->tau = tau0;
    c->knext = 0;
    c->stop = 0;
    c->status = TV_OK;
    c->n_active = n_active;
    c->seq = seq;
    c->t0 = c->t1 = 0;
    c->host_stop = host_stop;
}

// A resumed solve continues from the saved schedule position.
static __global__ void k_ctl_resume(SolveCtl *c, uint32_t *host_stop, uint32_t seq) {
    if (threadIdx.x != 0) return;
    c->stop = 0;
    c->status = TV_OK;
    c->seq = seq;
    c->t0 = c->t1 = 0;
    c->host_stop = host_stop;
}

// The accelerated schedule of the next `count` iterations (FP64, one thread;
// the same arithmetic as make_sched on the host).
static __global__ void k_ctl_sched(SolveCtl *c, IterSched *sc, int count) {
    if (threadIdx.x != 0 || c->stop) return;
    if (c->t0 == 0) c->t0 = wall_clock64();
    double tau = c->tau;
    for (int j = 0; j < count; ++j) {
        sc[j] = make_sched(tau, c->knext + j);
        tau *= sc[j].theta;
    }
    c->tau = tau;
    c->knext += count;
}

// Marks the solve stopped with `status` (one thread).
__device__ __forceinline__ void ctl_stop(SolveCtl *c, int status) {
    c->stop = 1;
    c->status = status;
    c->t1 = wall_clock64();
    if (c->host_stop) {
        *(volatile uint32_t *)c->host_stop = c->seq;
        __threadfence_system();
    }
}

// Milliseconds of device time since the first scheduled iteration, up to the
// stop (or now); clk_khz is the device wall clock's rate.
__device__ __forceinline__ double ctl_ms(const SolveCtl *c, double clk_khz) {
    if (c->t0 == 0 || clk_khz <= 0.0) return 0.0;
    const uint64_t t1 = c->stop ? c->t1 : wall_clock64();
    return (double)(t1 - c->t0) / clk_khz;
}

// Rate of the device wall clock in kHz (0 if unknown).
static inline double wall_clock_khz() {
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0.0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess) return 0.0;
    return (double)khz;
}

// The elementwise updates of the iteration, each rounded operation by
// operation as written (no multiply-add contraction, whichever kernel inlines
// them): the chain kernels' sources and sinks and the gap kernels then see the
// same bits for the same inputs in every build.
//
// b_i of the row step; shared by the row chain source and the gap kernel.
template <typename T>
__device__ __forceinline__ T row_data(T f, T x, T y, T tau, T inv1p) {
#pragma clang fp contract(off)
    return (tau * f + x - tau * y) * inv1p;
}
// eta_i = y_i + sigma xbar_i of the column step (its source and its sink).
template <typename T>
__device__ __forceinline__ T col_eta(T y, T sigma, T xb) {
#pragma clang fp contract(off)
    return y + sigma * xb;
}
// y'_i = eta_i - u_i (Moreau identity) of the column step's sink.
template <typename T>
__device__ __forceinline__ T col_dual(T y, T sigma, T xb, T u) {
#pragma clang fp contract(off)
    return col_eta<T>(y, sigma, xb) - u;
}
// xbar'_i = x'_i + theta (x'_i - x_i) of the row step's sink.
template <typename T>
__device__ __forceinline__ T row_xbar(T u, T theta, T x) {
#pragma clang fp contract(off)
    return u + theta * (u - x);
}
// The TV-l1 row step's chain data x_i - tau y_i.
template <typename T>
__device__ __forceinline__ T l1_row_data(T x, T tau, T y) {
#pragma clang fp contract(off)
    return x - tau * y;
}

// Store a clipped dual value in precision T, rounded toward zero so that the
// stored value still satisfies |p| <= lambda.
template <typename T> __device__ __forceinline__ T store_feasible(double p);
template <> __device__ __forceinline__ double store_feasible<double>(double p) { return p; }
template <> __device__ __forceinline__ float store_feasible<float>(double p) { return __double2float_rz(p); }

__device__ __forceinline__ double clipd(double v, double lam) { return v < -lam ? -lam : (v > lam ? lam : v); }

template <typename T>
__global__ __launch_bounds__(256) void k_fill(T *__restrict__ dst, int64_t n, T v) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) dst[i] = v;
}

// Copy between a dense H x W buffer and a strided one (leading dimension ld).
template <typename T>
__global__ __launch_bounds__(256) void k_copy2d(const T *__restrict__ src, int64_t lds, T *__restrict__ dst,
                                                int64_t ldd, int64_t H, int64_t W) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= H * W) return;
    const int64_t r = i / W, c = i % W;
    dst[r * ldd + c] = src[r * lds + c];
}

// Mean time of `reps` calls of fn after one untimed call (HIP events).
template <class Fn>
hipError_t time_calls(Fn fn, hipStream_t st, int reps, float *ms) {
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e != hipSuccess) return e;
    e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        hipEventDestroy(e0);
        return e;
    }
    e = fn();
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = fn();
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
    if (e == hipSuccess) *ms /= (float)reps;
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return e;
}

// Picks the fastest candidate plan of one launch; fills res.  G is the tag
// type of the launch's deque entries.
template <typename T, typename G = T, class Fn>
tv_status tune_launch(int64_t C, int64_t n, size_t seg_bytes, Fn launch, hipStream_t st, SegPlan *best_plan,
                             tv_tuning_result *res) {
    SegPlan cand[64];
    const int m = seg_candidates<T, G>(C, n, cand, 64);
    int best = -1, tried = 0;
    float best_ms = 0.0f;
    for (int j = 0; j < m; ++j) {
        if (seg_ws_bytes_plan<T, G>(C, n, cand[j]) > seg_bytes) continue;
        float ms = 0.0f;
        if (time_calls([&]() { return launch(cand[j]); }, st, 3, &ms) != hipSuccess) return TV_ERR_HIP;
        ++tried;
        if (best < 0 || ms < best_ms) {
            best = j;
            best_ms = ms;
        }
    }
    if (best < 0) return TV_ERR_WORKSPACE;
    *best_plan = cand[best];
    if (res) {
        res->segment_length = cand[best].L;
        res->halo = cand[best].H;
        res->ring_slots = cand[best].K;
        res->candidates = tried;
        res->ms = best_ms;
    }
    return TV_OK;
}

// Bounded lookahead of a solve's host loop (tv2d_options::lookahead = A > 0):
// after each chunk of iterations (one gap evaluation) the host records an
// event; before enqueuing chunk n it waits for the event of chunk n - A and
// reads the pinned host word that the device's stop writes this call's number
// to, and stops enqueuing once it is there.  The device keeps A - 1 chunks
// queued meanwhile, and a solve that stops early costs at most A chunks of
// launches that return at once.  The word and the events belong to the host
// thread and the device (one set per pair, kept until the process ends), so
// calls from one thread run their loops one after another; a call's number
// tells its stop from a late stop of an earlier call of the thread.
constexpr int kMaxLookahead = 64;
constexpr int kLookaheadDevices = 64;

struct StopMirror {
    uint32_t *host = nullptr;  // pinned host word
    uint32_t *dev = nullptr;   // its address on the device
    uint32_t seq = 0;
    hipEvent_t ev[kMaxLookahead] = {};
};

inline StopMirror *stop_mirror() {
    static thread_local StopMirror m[kLookaheadDevices];
    int d = 0;
    if (hipGetDevice(&d) != hipSuccess || d < 0 || d >= kLookaheadDevices) return nullptr;
    StopMirror &s = m[d];
    if (!s.host) {
        void *p = nullptr, *dp = nullptr;
        if (hipHostMalloc(&p, 256, hipHostMallocMapped | hipHostMallocPortable | hipHostMallocCoherent) !=
            hipSuccess)
            return nullptr;
        int made = 0;
        bool ok = hipHostGetDevicePointer(&dp, p, 0) == hipSuccess;
        while (ok && made < kMaxLookahead) {
            ok = hipEventCreateWithFlags(&s.ev[made], hipEventDisableTiming) == hipSuccess;
            if (ok) ++made;
        }
        if (!ok) {  // leave nothing half set up: a later call starts afresh
            for (int j = 0; j < made; ++j) (void)hipEventDestroy(s.ev[j]);
            (void)hipHostFree(p);
            return nullptr;
        }
        *(volatile uint32_t *)p = 0;
        s.host = (uint32_t *)p;
        s.dev = (uint32_t *)dp;
    }
    return &s;
}

struct Lookahead {
    StopMirror *m = nullptr;
    int depth = 0;
    uint32_t seq = 0;
    int n = 0;  // chunks enqueued
    // TV_OK, TV_ERR_INVALID_ARG when `st` is being captured into a graph (the
    // host cannot wait on work that does not run yet), or TV_ERR_HIP.
    tv_status begin(int lookahead, hipStream_t st) {
        depth = lookahead;
        if (depth <= 0) return TV_OK;
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(st, &cs) != hipSuccess) return TV_ERR_HIP;
        if (cs != hipStreamCaptureStatusNone) return TV_ERR_INVALID_ARG;
        m = stop_mirror();
        if (!m) return TV_ERR_HIP;
        seq = ++m->seq;
        if (seq == 0) seq = ++m->seq;  // 0 is never a call's number
        return TV_OK;
    }
    uint32_t *dev_word() const { return m ? m->dev : nullptr; }
    // Before enqueuing the next chunk: true once the device has stopped.
    bool stopped(hipError_t *err) {
        *err = hipSuccess;
        if (depth <= 0 || n < depth) return false;
        *err = hipEventSynchronize(m->ev[(n - depth) % depth]);
        return *err == hipSuccess && *(volatile uint32_t *)m->host == seq;
    }
    hipError_t chunk_done(hipStream_t st) {
        if (depth <= 0) return hipSuccess;
        return hipEventRecord(m->ev[n++ % depth], st);
    }
};

// Graphs of full chunks, one per starting parity, captured on a private
// stream on first use and replayed on the caller's stream.
struct ChunkGraphs {
    hipStream_t cap = nullptr;
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    bool failed = false;
    ~ChunkGraphs() {
        for (auto &x : exec)
            if (x) hipGraphExecDestroy(x);
        if (cap) hipStreamDestroy(cap);
    }
    template <class Fn>
    hipGraphExec_t get(int parity, Fn issue) {
        if (failed) return nullptr;
        if (exec[parity]) return exec[parity];
        if (!cap && hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) {
            failed = true;
            return nullptr;
        }
        hipGraph_t graph = nullptr;
        if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            failed = true;
            return nullptr;
        }
        const hipError_t e = issue(cap);
        const hipError_t e2 = hipStreamEndCapture(cap, &graph);
        if (e != hipSuccess || e2 != hipSuccess || !graph ||
            hipGraphInstantiate(&exec[parity], graph, nullptr, nullptr, 0) != hipSuccess) {
            exec[parity] = nullptr;
            failed = true;
        }
        if (graph) hipGraphDestroy(graph);
        return exec[parity];
    }
};

}  // namespace tvc
