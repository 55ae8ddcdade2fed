// Detailed-chemistry step on gfx950: one cell per lane, FP64 throughout.
//
// Each lane integrates the constant-pressure adiabatic reactor of its cell,
//   dY_k/dt = W_k wdot_k / rho,  dT/dt = -sum_k h_k dY_k/dt / cp
// (the species source term of the paper's Sec. "Chemistry Integration", with
// the density written out), with the L-stable Rosenbrock method RODAS4
// (Hairer & Wanner, Solving ODEs II, Sec. IV.7, transformed form) and an
// embedded error estimate.  The kernel is table-driven: the species and
// reaction tables live in one read-only allocation and are read with
// wave-uniform indices, so they arrive through the scalar cache as SGPR
// operands; per-lane state (y, Jacobian/LU, stage vectors) stays in
// registers.  Per-species arrays are indexed 1..K with index 0 a neutral
// element, so a reaction side with fewer than three molecules needs no
// branch.
#include <cmath>
#include <mutex>

#include "df_internal.h"
#include "df_kinetics.h"
#include "df_lane.h"

namespace df {
namespace {

template <int K>
__global__ __launch_bounds__(kWave) void chem_step_kernel(MechDev m, StepArgs a, const int32_t *__restrict__ cidx,
                                                       const int32_t *__restrict__ dcount) {
    using C = Cell<K>;
    __shared__ double lds[C::kRows * kWave];
    double *sh = lds + threadIdx.x;
    C::init_lds(sh);
    const int64_t slot = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t limit = dcount ? int64_t(*dcount) : a.n;
    if (slot >= limit) return;
    LaneTask<K> c;
    bool have = lane_load<K>(a, cidx ? int64_t(cidx[slot]) : slot, c);
    while (have) have = !lane_attempt<K>(m, a, sh, c);
}

}  // namespace
}  // namespace df

namespace df {

template <int K>
static df_status launch_k(const MechDev &m, const StepArgs &a, const int32_t *cidx, const int32_t *dcount,
                          hipStream_t stream) {
    const int64_t blocks = (a.n + 63) / 64;
    hipLaunchKernelGGL(chem_step_kernel<K>, dim3(unsigned(blocks)), dim3(64), 0, stream, m, a, cidx, dcount);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(DF_E_HIP, std::string("chem_step launch: ") + hipGetErrorString(e));
    return DF_OK;
}

df_status launch_chem_step(const MechDev &m, const StepArgs &a, int mapping, const int32_t *cidx,
                           const int32_t *dcount, hipStream_t stream) {
    if (a.n == 0) return DF_OK;
    // mapping 0 picks 16 lanes per cell whenever a kernel is compiled for K: one sub-step
    // then takes a fraction of the latency, which bounds a stiff cell's step time; with the cost
    // order (and reaction slots that divide in two) the head of the order takes 32 lanes, the
    // head variant (mapping 5), whose stiffest cells then finish sooner
    if (mapping == 3) return launch_chem_wave(m, a, cidx, dcount, stream);
    if (mapping == 2 || mapping == 4 || mapping == 5 || (mapping == 0 && chem_coop_supported(m)))
        return launch_chem_coop(m, a, CellQueue{cidx, dcount, nullptr, nullptr, nullptr, 0}, stream,
                                mapping == 4 ? 2 : (mapping == 5 || mapping == 0 ? 3 : 1));
    if (a.n > int64_t(64) * 0x7fffffff) return fail(DF_E_UNSUPPORTED, "df_chem_step: too many cells for one launch");
    switch (m.K) {
#define DF_CASE(k) \
    case k:        \
        return launch_k<k>(m, a, cidx, dcount, stream);
        DF_CHEM_SPECIES_LIST(DF_CASE)
#undef DF_CASE
        default:
            if (mapping == 0 && chem_wave_supported(m)) return launch_chem_wave(m, a, cidx, dcount, stream);
            return fail(DF_E_UNSUPPORTED, "df_chem_step: no compiled kernel for " + std::to_string(m.K) + " species");
    }
}

// ---- cost ordering: counting sort of the cells on (temperature, step length) buckets ----
namespace {

constexpr int kTB = 256, kDB = 16;      // temperature and step-length buckets
constexpr int kBuckets = kTB * kDB;     // bucket = tb * kDB + db; bucket 0 = hottest, longest step
constexpr double kTlo = 200.0, kThi = 3500.0;
constexpr int kOrdThreads = 256;
// cells of the buckets at or below about this temperature form the cold tail of the queue,
// the only cells one-cell-per-lane waves take (they need about one sub-step each)
constexpr double kTcold = 500.0;

// hottest first; non-finite temperatures go last
__device__ __forceinline__ int t_bucket(double T) {
    if (!(T == T) || !isfinite(T)) return kTB - 1;
    const double x = (kThi - T) * (double(kTB) / (kThi - kTlo));
    return int(fmin(fmax(x, 0.0), double(kTB - 1)));
}

// longest step first: four buckets per decade below 1 ms; non-positive or non-finite last
__device__ __forceinline__ int d_bucket(double dt) {
    if (!(dt > 0.0) || !isfinite(dt)) return kDB - 1;
    const double x = 4.0 * log10(1e-3 / dt);
    return int(fmin(fmax(x, 0.0), double(kDB - 1)));
}

__device__ __forceinline__ int cost_bucket(const double *T, const double *dts, double dt, int64_t i) {
    return t_bucket(T[i]) * kDB + d_bucket(dts ? dts[i] : dt);
}

// zero the bucket counts and the queue counter
__global__ __launch_bounds__(kOrdThreads) void order_zero(int32_t *cnt, unsigned long long *ctr) {
    for (int b = threadIdx.x; b < 2 * kBuckets; b += kOrdThreads) cnt[b] = 0;
    if (threadIdx.x == 0) *ctr = 0ull;
}

__global__ __launch_bounds__(kOrdThreads) void order_hist(const double *__restrict__ T, const double *__restrict__ dts,
                                                          double dt, int64_t n, int32_t *__restrict__ cnt) {
    __shared__ int32_t loc[kBuckets];
    for (int b = threadIdx.x; b < kBuckets; b += kOrdThreads) loc[b] = 0;
    __syncthreads();
    const int64_t i = int64_t(blockIdx.x) * kOrdThreads + threadIdx.x;
    if (i < n) atomicAdd(&loc[cost_bucket(T, dts, dt, i)], 1);
    __syncthreads();
    for (int b = threadIdx.x; b < kBuckets; b += kOrdThreads)
        if (loc[b]) atomicAdd(&cnt[b], loc[b]);
}

// exclusive scan of the bucket counts into the second half of cnt (one block: each thread
// scans a run of kBuckets / kOrdThreads buckets, then the run totals are scanned); also the
// number of cells in the cold buckets, at cnt[2 * kBuckets]
__global__ __launch_bounds__(kOrdThreads) void order_scan(int32_t *cnt) {
    constexpr int R = kBuckets / kOrdThreads;
    __shared__ int32_t v[kOrdThreads];
    const int t = threadIdx.x;
    int32_t run = 0;
    for (int q = 0; q < R; ++q) run += cnt[t * R + q];
    v[t] = run;
    __syncthreads();
    for (int off = 1; off < kOrdThreads; off <<= 1) {
        const int32_t add = (t >= off) ? v[t - off] : 0;
        __syncthreads();
        v[t] += add;
        __syncthreads();
    }
    int32_t base = v[t] - run;
    const int32_t total = v[kOrdThreads - 1];
    const int bcold = t_bucket(kTcold) * kDB;
    for (int q = 0; q < R; ++q) {
        if (t * R + q == bcold) cnt[2 * kBuckets] = total - base;
        cnt[kBuckets + t * R + q] = base;
        base += cnt[t * R + q];
    }
}

__global__ __launch_bounds__(kOrdThreads) void order_scatter(const double *__restrict__ T,
                                                             const double *__restrict__ dts, double dt, int64_t n,
                                                             int32_t *__restrict__ cnt, int32_t *__restrict__ idx) {
    __shared__ int32_t loc[kBuckets], base[kBuckets];
    for (int b = threadIdx.x; b < kBuckets; b += kOrdThreads) loc[b] = 0;
    __syncthreads();
    const int64_t i = int64_t(blockIdx.x) * kOrdThreads + threadIdx.x;
    int b = 0, rank = 0;
    if (i < n) {
        b = cost_bucket(T, dts, dt, i);
        rank = atomicAdd(&loc[b], 1);
    }
    __syncthreads();
    for (int q = threadIdx.x; q < kBuckets; q += kOrdThreads)
        if (loc[q]) base[q] = atomicAdd(&cnt[kBuckets + q], loc[q]);
    __syncthreads();
    if (i < n) idx[base[b] + rank] = int32_t(i);
}

constexpr size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

// workspace: bucket counts and offsets | queue counter | cell order
constexpr size_t kCntBytes = size_t(2 * kBuckets + 64) * 4;
constexpr size_t order_bytes(int64_t n) { return al256(kCntBytes) + 256 + al256(size_t(n) * 4); }

struct Work {
    int32_t *cnt;
    unsigned long long *ctr;
    int32_t *idx;
    int32_t *tail;  // cells in the cold buckets
};

Work work_parts(void *ws) {
    auto *b = static_cast<unsigned char *>(ws);
    auto *cnt = reinterpret_cast<int32_t *>(b);
    return Work{cnt, reinterpret_cast<unsigned long long *>(b + al256(kCntBytes)),
                reinterpret_cast<int32_t *>(b + al256(kCntBytes) + 256), cnt + 2 * kBuckets};
}

// cells in order of decreasing estimated cost into w.idx; zeroes the queue counter
df_status order_cells(const StepArgs &a, const Work &w, hipStream_t s) {
    const unsigned blocks = unsigned((a.n + kOrdThreads - 1) / kOrdThreads);
    hipLaunchKernelGGL(order_zero, dim3(1), dim3(kOrdThreads), 0, s, w.cnt, w.ctr);
    hipLaunchKernelGGL(order_hist, dim3(blocks), dim3(kOrdThreads), 0, s, a.T, a.dts, a.dt, a.n, w.cnt);
    hipLaunchKernelGGL(order_scan, dim3(1), dim3(kOrdThreads), 0, s, w.cnt);
    hipLaunchKernelGGL(order_scatter, dim3(blocks), dim3(kOrdThreads), 0, s, a.T, a.dts, a.dt, a.n, w.cnt, w.idx);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(DF_E_HIP, std::string("df_chem_step ordering: ") + hipGetErrorString(e));
    return DF_OK;
}

// scalar dt (dts == nullptr) or per-cell dt
df_status chem_step_impl(const char *who, const df_mech *mech, int64_t n_cells, int64_t ld, double dt,
                         const double *dts, const double *p, double *T, double *Y, double *h_inout, double *rr,
                         int32_t *cell_status, int32_t *n_steps, void *workspace, size_t ws_bytes,
                         const df_chem_opts *opts, void *hip_stream) {
    const std::string w(who);
    if (!mech) return fail(DF_E_INVALID, w + ": null mechanism handle");
    if (n_cells < 0 || ld < n_cells) return fail(DF_E_INVALID, w + ": need 0 <= n_cells <= ld");
    if (!dts && (!(dt > 0.0) || !std::isfinite(dt))) return fail(DF_E_INVALID, w + ": dt must be finite and > 0");
    if (n_cells > 0 && (!p || !T || !Y)) return fail(DF_E_INVALID, w + ": null p, T or Y");
    if (n_cells > 0x7fffffff) return fail(DF_E_UNSUPPORTED, w + ": more than 2^31-1 cells");
    df_chem_opts o;
    df_chem_default_opts(&o);
    if (opts) o = *opts;
    df_status st = validate_chem_opts(o);
    if (st != DF_OK) return st;
    if (workspace && (ws_bytes < order_bytes(n_cells) || reinterpret_cast<uintptr_t>(workspace) % 256 != 0))
        return fail(DF_E_INVALID, w + ": workspace smaller than df_chem_workspace_size or not 256-byte aligned");
    if (o.schedule == 2 && !workspace) return fail(DF_E_INVALID, w + ": the queue schedule needs the workspace");
    if (n_cells == 0) return DF_OK;
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess) return fail(DF_E_HIP, w + ": hipGetDevice failed");
    if (prev != mech->device && hipSetDevice(mech->device) != hipSuccess)
        return fail(DF_E_HIP, w + ": cannot select the mechanism's device");
    auto s = static_cast<hipStream_t>(hip_stream);
    const StepArgs a{n_cells, ld, dt, dts, p, T, Y, h_inout, rr, cell_status, n_steps, kernel_opts(o), DF_CELL_OK};
    const Work wk = workspace ? work_parts(workspace) : Work{nullptr, nullptr, nullptr, nullptr};
    if (workspace) st = order_cells(a, wk, s);
    if (st == DF_OK) {
        if (o.schedule == 2) {
            const int32_t cap = chem_queue_capacity(mech->dev);
            int32_t head = o.coop_blocks == 0 ? cap : (o.coop_blocks < 0 ? 0 : o.coop_blocks);
            head = head > cap ? cap : head;
            if (cap <= 0)
                st = fail(DF_E_UNSUPPORTED, w + ": no persistent kernel for this mechanism");
            else
                st = launch_chem_queue(mech->dev, a, CellQueue{nullptr, nullptr, wk.idx, wk.ctr, wk.tail, head}, cap,
                                       s);
        } else {
            st = launch_chem_step(mech->dev, a, o.mapping, workspace ? wk.idx : nullptr, nullptr, s);
        }
    }
    if (prev != mech->device) (void)hipSetDevice(prev);
    return st;
}

}  // namespace

}  // namespace df

extern "C" df_status df_chem_workspace_size(const df_mech *mech, int64_t n_cells, size_t *bytes) {
    using namespace df;
    clear_error();
    if (!mech || !bytes || n_cells < 0) return fail(DF_E_INVALID, "df_chem_workspace_size: bad arguments");
    *bytes = order_bytes(n_cells);
    return DF_OK;
}

extern "C" df_status df_chem_step(const df_mech *mech, int64_t n_cells, int64_t ld, double dt, const double *p,
                                  double *T, double *Y, double *h_inout, double *rr, int32_t *cell_status,
                                  int32_t *n_steps, void *workspace, size_t ws_bytes, const df_chem_opts *opts,
                                  void *hip_stream) {
    df::clear_error();
    return df::chem_step_impl("df_chem_step", mech, n_cells, ld, dt, nullptr, p, T, Y, h_inout, rr, cell_status,
                              n_steps, workspace, ws_bytes, opts, hip_stream);
}

extern "C" df_status df_chem_step_cells(const df_mech *mech, int64_t n_cells, int64_t ld, const double *dt,
                                        const double *p, double *T, double *Y, double *h_inout, double *rr,
                                        int32_t *cell_status, int32_t *n_steps, void *workspace, size_t ws_bytes,
                                        const df_chem_opts *opts, void *hip_stream) {
    df::clear_error();
    if (n_cells > 0 && !dt) return df::fail(DF_E_INVALID, "df_chem_step_cells: null dt");
    return df::chem_step_impl("df_chem_step_cells", mech, n_cells, ld, 0.0, dt, p, T, Y, h_inout, rr, cell_status,
                              n_steps, workspace, ws_bytes, opts, hip_stream);
}

// ---- the step without a caller workspace: the cost-ordering scratch in a static device array ----
namespace df {
namespace {

// Cells one call of df_chem_step_noalloc takes at most; its scratch holds the bucket counts, the
// queue counter and the cell order of that many cells (4 bytes a cell, 4.2 MB in all), in every
// device's copy of the code object until the process ends.
constexpr int64_t kNoAllocMaxCells = int64_t(1) << 20;
constexpr size_t kNoAllocBytes = order_bytes(kNoAllocMaxCells);

__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

// the device address of each device's copy of `scratch`, taken once per device with that device
// current (the array's name is not a device address in host code)
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

df_status scratch_on(int device, void **out) {
    if (device < 0 || device >= kMaxDevices) return fail(DF_E_UNSUPPORTED, "df_chem_step_noalloc: device index beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(DF_E_HIP, std::string("df_chem_step_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e));
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return DF_OK;
}

}  // namespace
}  // namespace df

extern "C" df_status df_chem_step_noalloc(const df_mech *mech, int64_t n_cells, int64_t ld, double dt,
                                          const double *p, double *T, double *Y, double *h_inout, double *rr,
                                          int32_t *cell_status, int32_t *n_steps, const df_chem_opts *opts,
                                          void *hip_stream) {
    using namespace df;
    clear_error();
    const char *who = "df_chem_step_noalloc";
    if (!mech) return fail(DF_E_INVALID, std::string(who) + ": null mechanism handle");
    if (n_cells > kNoAllocMaxCells)
        return fail(DF_E_UNSUPPORTED, std::string(who) + ": " + std::to_string(n_cells) + " cells, at most " +
                                          std::to_string(kNoAllocMaxCells) + " per call");
    if (n_cells <= 0) return chem_step_impl(who, mech, n_cells, ld, dt, nullptr, p, T, Y, h_inout, rr, cell_status,
                                            n_steps, nullptr, 0, opts, hip_stream);
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess) return fail(DF_E_HIP, std::string(who) + ": hipGetDevice failed");
    if (prev != mech->device && hipSetDevice(mech->device) != hipSuccess)
        return fail(DF_E_HIP, std::string(who) + ": cannot select the mechanism's device");
    void *ws = nullptr;
    df_status st = scratch_on(mech->device, &ws);
    if (prev != mech->device) (void)hipSetDevice(prev);
    if (st != DF_OK) return st;
    return chem_step_impl(who, mech, n_cells, ld, dt, nullptr, p, T, Y, h_inout, rr, cell_status, n_steps, ws,
                          order_bytes(n_cells), opts, hip_stream);
}

// ---- schedule autotuning ----
namespace df {
namespace {

size_t autotune_bytes(int K, int64_t n) {
    return order_bytes(n) + al256(size_t(n) * 8) + al256(size_t(K) * size_t(n) * 8);
}

}  // namespace
}  // namespace df

extern "C" df_status df_chem_autotune_workspace_size(const df_mech *mech, int64_t n_cells, size_t *bytes) {
    using namespace df;
    clear_error();
    if (!mech || !bytes || n_cells < 0) return fail(DF_E_INVALID, "df_chem_autotune_workspace_size: bad arguments");
    *bytes = autotune_bytes(mech->host.K, n_cells);
    return DF_OK;
}

extern "C" df_status df_chem_autotune(const df_mech *mech, int64_t n_cells, int64_t ld, double dt,
                                      const double *dt_cells, const double *p, const double *T, const double *Y,
                                      void *workspace, size_t ws_bytes, df_chem_opts *opts, void *hip_stream) {
    using namespace df;
    clear_error();
    const char *who = "df_chem_autotune";
    if (!mech || !opts) return fail(DF_E_INVALID, std::string(who) + ": null mechanism handle or opts");
    if (n_cells < 0 || ld < n_cells) return fail(DF_E_INVALID, std::string(who) + ": need 0 <= n_cells <= ld");
    if (!dt_cells && (!(dt > 0.0) || !std::isfinite(dt)))
        return fail(DF_E_INVALID, std::string(who) + ": dt must be finite and > 0");
    if (n_cells > 0 && (!p || !T || !Y)) return fail(DF_E_INVALID, std::string(who) + ": null p, T or Y");
    df_status st = validate_chem_opts(*opts);
    if (st != DF_OK) return st;
    const int K = mech->host.K;
    if (!workspace || ws_bytes < autotune_bytes(K, n_cells) || reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
        return fail(DF_E_INVALID, std::string(who) + ": workspace smaller than df_chem_autotune_workspace_size or "
                                                     "not 256-byte aligned");
    if (n_cells == 0) return DF_OK;
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess) return fail(DF_E_HIP, std::string(who) + ": hipGetDevice failed");
    if (prev != mech->device && hipSetDevice(mech->device) != hipSuccess)
        return fail(DF_E_HIP, std::string(who) + ": cannot select the mechanism's device");
    auto s = static_cast<hipStream_t>(hip_stream);
    auto *base = static_cast<unsigned char *>(workspace);
    void *ows = base;
    auto *Tc = reinterpret_cast<double *>(base + order_bytes(n_cells));
    auto *Yc = reinterpret_cast<double *>(base + order_bytes(n_cells) + al256(size_t(n_cells) * 8));
    const int32_t cap = chem_queue_capacity(mech->dev);
    struct Cand {
        int32_t schedule, coop_blocks, mapping;
    };
    std::vector<Cand> cands = {{1, 0, opts->mapping}};
    if (chem_coop_supported(mech->dev) && mech->dev.RPL % 2 == 0 && (opts->mapping == 0 || opts->mapping == 2))
        cands.push_back({1, 0, 4});
    // one cell per lane: 64 cells per wave, for fields where the total work, not one cell's chain
    // of sub-steps, sets the time
    bool lane_kernel = false;
    switch (K) {
#define DF_CASE(k)         \
    case k:                \
        lane_kernel = true; \
        break;
        DF_CHEM_SPECIES_LIST(DF_CASE)
#undef DF_CASE
        default:
            break;
    }
    if (lane_kernel && (opts->mapping == 0 || opts->mapping == 2)) cands.push_back({1, 0, 1});
    if (cap > 0) {
        cands.push_back({2, 0, opts->mapping});
        cands.push_back({2, cap / 2, opts->mapping});
        cands.push_back({2, (3 * cap) / 4, opts->mapping});
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float best_ms = -1.0f;
    Cand best = cands[0];
    hipError_t he = hipEventCreate(&e0);
    if (he == hipSuccess) he = hipEventCreate(&e1);
    for (size_t c = 0; c < cands.size() && he == hipSuccess && st == DF_OK; ++c) {
        df_chem_opts o = *opts;
        o.schedule = cands[c].schedule;
        o.coop_blocks = cands[c].coop_blocks;
        o.mapping = cands[c].mapping;
        for (int rep = 0; rep < 2 && he == hipSuccess && st == DF_OK; ++rep) {
            he = hipMemcpyAsync(Tc, T, size_t(n_cells) * 8, hipMemcpyDeviceToDevice, s);
            if (he == hipSuccess)
                he = hipMemcpy2DAsync(Yc, size_t(n_cells) * 8, Y, size_t(ld) * 8, size_t(n_cells) * 8, size_t(K),
                                      hipMemcpyDeviceToDevice, s);
            if (he == hipSuccess) he = hipEventRecord(e0, s);
            if (he != hipSuccess) break;
            st = chem_step_impl(who, mech, n_cells, n_cells, dt, dt_cells, p, Tc, Yc, nullptr, nullptr, nullptr,
                                nullptr, ows, order_bytes(n_cells), &o, hip_stream);
            if (st != DF_OK) break;
            he = hipEventRecord(e1, s);
            if (he == hipSuccess) he = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
            if (he == hipSuccess && (best_ms < 0.0f || ms < best_ms)) {
                best_ms = ms;
                best = cands[c];
            }
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (prev != mech->device) (void)hipSetDevice(prev);
    if (st != DF_OK) return st;
    if (he != hipSuccess) return fail(DF_E_HIP, std::string(who) + ": " + hipGetErrorString(he));
    opts->schedule = best.schedule;
    opts->coop_blocks = best.coop_blocks;
    opts->mapping = best.mapping;
    return DF_OK;
}
