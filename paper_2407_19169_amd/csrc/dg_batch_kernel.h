// dg_batch_kernel.h — many independent 1D problems of different size and
// degree in one persistent launch (gfx950).
//
// Each workgroup pulls whole problems from an atomic queue (the host orders
// the queue longest-first, by cost n (k+1)^2 steps) and advances each one
// through all of its time steps on its own: a CFL reduction over the
// workgroup, then one pass over the problem's tiles that runs all three
// SSP-RK3 stages (with the filter after each) of a tile of BS - 12 cells
// (BS = 128 or 256 threads, a choice of the autotuner) and its 6-cell halo.  No grid-wide synchronisation is needed: a problem never
// leaves its workgroup.
// (included at the end of dg1d.hip: it reuses the 1D tile function)
#include "dg_batch.h"

namespace dg {

namespace {

template <int BS>
__device__ __forceinline__ double block_max(double v, double* red)
{
    v = wave_max(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double r = red[0];
#pragma unroll
    for (int i = 1; i < BS / 64; ++i) r = (red[i] > r || red[i] != red[i]) ? red[i] : r;
    __syncthreads();
    return r;
}

// Deterministic block sum: fixed strided partial sums, fixed-order tree.
template <int BS>
__device__ __forceinline__ double block_sum(double v, double* tree)
{
    tree[threadIdx.x] = v;
    __syncthreads();
    for (int w = BS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) tree[threadIdx.x] += tree[threadIdx.x + w];
        __syncthreads();
    }
    const double r = tree[0];
    __syncthreads();
    return r;
}

template <typename TB>
__device__ __forceinline__ StateView<TB> prob_view(void* base, const BatchProb& p, int k)
{
    StateView<TB> v;
    unsigned char* b = static_cast<unsigned char*>(base) + p.off_int;
    v.m0 = reinterpret_cast<double*>(b);
    v.s0 = p.n_pad;
    v.hi = reinterpret_cast<TB*>(v.m0 + 3 * p.n_pad);
    v.sv = (int64_t)k * p.n_pad;
    v.sl = p.n_pad;
    return v;
}

template <int K, typename TB, int MODE, int PP, int BS>
__device__ __forceinline__ void solve_problem(const BatchArgs& b, const BatchProb& pr, unsigned int pidx,
                              unsigned char* lds, double* red, double* tree, double* sflux,
                              int* sreject)
{
    // the step's three stages in one pass: each consumes a halo of 1 (no
    // filter) or 2 (filter) cells per side
    constexpr int TILE3 = BS - 2 * 3 * (MODE == 0 ? 1 : 2);
    StateView<TB> A = prob_view<TB>(b.u[0], pr, K);
    StateView<TB> B = prob_view<TB>(b.u[1], pr, K);
    const StateView<TB> A0 = A, B0 = B;
    Ctrl* ctrl = &b.ctrl[pidx];
    const int64_t n = pr.n;
    const int64_t ntiles3 = (n + TILE3 - 1) / TILE3;

    Args1D<TB> a;
    a.n = n;
    a.inv_h = pr.inv_h;
    a.periodic = pr.bc_lo == BC_PERIODIC;
    a.bc_lo = pr.bc_lo;
    a.bc_hi = pr.bc_hi;
#pragma unroll
    for (int v = 0; v < 4; ++v) a.dir_lo[v] = a.dir_hi[v] = 0.0;
    a.phys = b.phys;
    a.dt_from_ctrl = 0;
    a.check = 1;
    a.ctrl = ctrl;
    a.bflux = sflux;
    a.alpha_acc = nullptr;
    a.eta_acc = nullptr;
    a.tcount = nullptr;
    a.tcell = nullptr;
    a.tdata = nullptr;
    a.E_out = nullptr;
    a.eta_out = nullptr;
    a.pp = PP;  // compile-time, so the limiter's code exists only where it runs
    a.reject = sreject;

    // CFL quantity of the initial state
    double lam = 0.0;
    for (int64_t c = threadIdx.x; c < n; c += BS) {
        double ub[3];
#pragma unroll
        for (int v = 0; v < 3; ++v) ub[v] = A.m0[v * A.s0 + c];
        const double l = Phys1D<EULER>::speed(ub, b.phys);
        lam = (l > lam || l != l) ? l : lam;
    }
    double alpha = block_max<BS>(lam, red);

    double t = 0.0, dtmin = INFINITY, dtmax = 0.0;
    double bfl[3] = {0.0, 0.0, 0.0};
    long long steps = 0, restarts = 0;
    int retries = 0;
    const double t_end = pr.t_end;
    double dt = 0.0;
    bool last = false, retry = false;
    while (steps < b.steps && t < t_end) {
        if (ctrl->status == -4) break;  // non-finite: stop; positivity: report only
        if (!retry) {
            dt = b.cfl * pr.h / alpha;
            // a non-finite step, or one too small to advance t, ends the run
            if (!(dt > 0.0) || !isfinite(dt) || !(t + dt > t)) {
                if (threadIdx.x == 0) latch_error(ctrl, -4, -1);
                break;
            }
            last = false;
            if (t + dt >= t_end) {
                dt = t_end - t;
                last = true;
            }
        }
        retry = false;
        double net[3] = {0.0, 0.0, 0.0};
        {
            // the whole step in one pass over the problem's tiles (6-cell
            // halo): u^n (A) -> u^{n+1} (B), stages in registers and LDS
            a.un = a.us = A;
            a.out = B;
            a.stage = 2;
            a.want_lam = true;
            if (threadIdx.x < 24) sflux[threadIdx.x] = 0.0;
            if (threadIdx.x == 0) *sreject = 0;
            __syncthreads();
            double lmax = 0.0;
            for (int64_t tile = 0; tile < ntiles3; ++tile) {
                double l, e;
                stage1d_tile<EULER, K, TB, MODE, BS, false, 3>(a, tile, dt, lds, &l, &e);
                lmax = (l > lmax || l != l) ? l : lmax;
                __syncthreads();  // the next tile reuses the LDS
            }
            if (*sreject) {
                // positivity limiter: a stage left an inadmissible cell
                // average; u^n (buffer A) is untouched, so the step is
                // simply run again with half the time step
                retry = true;
            } else {
#pragma unroll
                for (int s = 0; s < 3; ++s)
#pragma unroll
                    for (int v = 0; v < 3; ++v)
                        net[v] += kStageWeight[s] * (sflux[8 * s + 4 + v] - sflux[8 * s + v]);
                alpha = block_max<BS>(lmax, red);
            }
        }
        if (retry) {
            __syncthreads();  // every lane has read the flag before it is cleared
            if (++retries > kMaxRetries) {
                if (threadIdx.x == 0) latch_error(ctrl, -5, -1);
                break;
            }
            ++restarts;
            dt *= 0.5;
            last = false;
            continue;
        }
        retries = 0;
#pragma unroll
        for (int v = 0; v < 3; ++v) bfl[v] += dt * net[v];
        t = last ? t_end : t + dt;
        ++steps;
        dtmin = dt < dtmin ? dt : dtmin;
        dtmax = dt > dtmax ? dt : dtmax;
        const StateView<TB> tmp = A;  // the step's output is in B
        A = B;
        B = tmp;
    }
    if (steps & 1) {
        // the solution sits in the second buffer: copy it to the first
        for (int64_t c = threadIdx.x; c < n; c += BS)
#pragma unroll
            for (int v = 0; v < 3; ++v) {
                A0.m0[v * A0.s0 + c] = B0.m0[v * B0.s0 + c];
#pragma unroll
                for (int l = 1; l <= K; ++l)
                    A0.hi[v * A0.sv + (l - 1) * A0.sl + c] = B0.hi[v * B0.sv + (l - 1) * B0.sl + c];
            }
        __syncthreads();
    }
    // FP64 ledger of the final state
    double led[3];
#pragma unroll
    for (int v = 0; v < 3; ++v) {
        double acc = 0.0;
        for (int64_t c = threadIdx.x; c < n; c += BS) acc += A0.m0[v * A0.s0 + c];
        led[v] = pr.h * block_sum<BS>(acc, tree);
    }
    if (threadIdx.x == 0) {
        BatchReport& r = b.report[pidx];
        r.steps = steps;
        r.t = t;
        r.dt_min = dtmin;
        r.dt_max = dtmax;
        for (int v = 0; v < 3; ++v) {
            r.ledger[v] = led[v];
            r.bflux[v] = bfl[v];
        }
        r.status = ctrl->status;
        r.first_bad = ctrl->first_bad;
        r.restarts = restarts;
    }
}

template <typename TB, int MODE, int BS>
struct BatchLds {
    static constexpr int a = Stage1DLds<EULER, 0, TB, MODE, BS>::bytes;
    static constexpr int b = Stage1DLds<EULER, 1, TB, MODE, BS>::bytes;
    static constexpr int c = Stage1DLds<EULER, 2, TB, MODE, BS>::bytes;
    static constexpr int d = Stage1DLds<EULER, 3, TB, MODE, BS>::bytes;
    static constexpr int ab = a > b ? a : b;
    static constexpr int cd = c > d ? c : d;
    static constexpr int bytes = ab > cd ? ab : cd;
};

}  // namespace

// Register budget of the mixed form: 3 waves per SIMD (168 VGPRs; its LDS
// allows 4 workgroups per CU) without the positivity limiter, 2 with it (a
// budget of 3 spills, and measured slower).  The FP64 form is left free.
template <typename TB, int PP>
struct BatchWaves {
    static constexpr int value = sizeof(TB) == 4 ? 3 : 1;
};

template <typename TB, int MODE, int PP, int BS>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(BatchWaves<TB, PP>::value)))
void batch1d_kernel(BatchArgs b)
{
    __shared__ __align__(16) unsigned char lds[BatchLds<TB, MODE, BS>::bytes];
    __shared__ double red[BS / 64];
    __shared__ double tree[BS];
    __shared__ double sflux[24];  // boundary fluxes, lo[4] hi[4] per stage
    __shared__ int sreject;
    __shared__ unsigned int s_pi;
    for (;;) {
        if (threadIdx.x == 0) s_pi = atomicAdd(b.queue, 1u);
        __syncthreads();
        const unsigned int pi = s_pi;
        __syncthreads();
        if (pi >= (unsigned int)b.nprob) break;
        const unsigned int p = b.order[pi];
        const BatchProb pr = b.probs[p];
        switch (pr.k) {
        case 0: solve_problem<0, TB, MODE, PP, BS>(b, pr, p, lds, red, tree, sflux, &sreject); break;
        case 1: solve_problem<1, TB, MODE, PP, BS>(b, pr, p, lds, red, tree, sflux, &sreject); break;
        case 2: solve_problem<2, TB, MODE, PP, BS>(b, pr, p, lds, red, tree, sflux, &sreject); break;
        default: solve_problem<3, TB, MODE, PP, BS>(b, pr, p, lds, red, tree, sflux, &sreject); break;
        }
        __syncthreads();
    }
}

// Start of a batched run: the queue head and every problem's error latch
// cleared (a kernel, so the run can be captured in a graph).
__global__ __launch_bounds__(256) void batch_reset_kernel(unsigned int* queue, Ctrl* ctrl, int nprob)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i == 0) *queue = 0u;
    if (i < nprob) {
        ctrl[i].status = 0;
        ctrl[i].first_bad = -1;
        ctrl[i].reject = 0;
    }
}

// FP64 exchange layout (problems packed back to back, [var][mode][cell])
// <-> the internal per-problem blocks; one workgroup per problem.
template <typename TB>
__global__ __launch_bounds__(256) void batch_convert_kernel(int to_internal, BatchArgs b, double* ext)
{
    const BatchProb pr = b.probs[blockIdx.x];
    const StateView<TB> v = prob_view<TB>(b.u[0], pr, pr.k);
    const int K1 = pr.k + 1;
    const long long total = 3LL * K1 * pr.n;
    for (long long i = threadIdx.x; i < total; i += 256) {
        const long long c = i % pr.n;
        const int l = (int)((i / pr.n) % K1);
        const int var = (int)(i / (pr.n * K1));
        double* e = ext + pr.off_ext + i;
        if (l == 0) {
            double* p = v.m0 + var * v.s0 + c;
            if (to_internal)
                *p = *e;
            else
                *e = *p;
        } else {
            TB* p = v.hi + var * v.sv + (long long)(l - 1) * v.sl + c;
            if (to_internal)
                *p = (TB)*e;
            else
                *e = (double)*p;
        }
    }
}

template <typename TB>
hipError_t launch_batch_convert(int to_internal, const BatchArgs& b, const double* ext, int nprob,
                                hipStream_t st)
{
    hipLaunchKernelGGL((batch_convert_kernel<TB>), dim3(nprob), dim3(256), 0, st, to_internal, b,
                       const_cast<double*>(ext));
    return hipGetLastError();
}
template hipError_t launch_batch_convert<double>(int, const BatchArgs&, const double*, int, hipStream_t);
template hipError_t launch_batch_convert<float>(int, const BatchArgs&, const double*, int, hipStream_t);

template <typename TB, int BS>
static void launch_batch_tb(int mode, const BatchArgs& b, int grid, hipStream_t st)
{
    if (mode == 0 && !b.pp)
        hipLaunchKernelGGL((batch1d_kernel<TB, 0, 0, BS>), dim3(grid), dim3(BS), 0, st, b);
    else if (mode == 0)
        hipLaunchKernelGGL((batch1d_kernel<TB, 0, 1, BS>), dim3(grid), dim3(BS), 0, st, b);
    else if (!b.pp)
        hipLaunchKernelGGL((batch1d_kernel<TB, 1, 0, BS>), dim3(grid), dim3(BS), 0, st, b);
    else
        hipLaunchKernelGGL((batch1d_kernel<TB, 1, 1, BS>), dim3(grid), dim3(BS), 0, st, b);
}

hipError_t launch_batch1d(int mixed, int mode, const BatchArgs& b, int grid, int bs, hipStream_t st)
{
    if (bs != 128 && bs != 256) return hipErrorInvalidValue;
    if (mixed)
        bs == 128 ? launch_batch_tb<float, 128>(mode, b, grid, st) : launch_batch_tb<float, 256>(mode, b, grid, st);
    else
        bs == 128 ? launch_batch_tb<double, 128>(mode, b, grid, st) : launch_batch_tb<double, 256>(mode, b, grid, st);
    return hipGetLastError();
}

hipError_t launch_batch_reset(const BatchArgs& b, hipStream_t st)
{
    const unsigned g = (unsigned)((b.nprob + 255) / 256);
    hipLaunchKernelGGL(batch_reset_kernel, dim3(g < 1 ? 1 : g), dim3(256), 0, st, b.queue, b.ctrl, b.nprob);
    return hipGetLastError();
}

}  // namespace dg
