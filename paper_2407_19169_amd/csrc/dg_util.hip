// dg_util.hip — time-step control, layout conversion, conservation ledger
// and state checks shared by the 1D and 2D paths.
#include "dg_kernels.h"

namespace dg {

// One thread; runs between the stage kernels.  The control block is read
// into registers in one burst of loads, updated there and written back, so
// its dependent branches cost no memory round trips.
__global__ void step_ctrl_kernel(Ctrl* c, int finalize_only)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    CtrlRegs r = load_ctrl_regs<false>(c);
    step_ctrl_body(&r, finalize_only);
    store_ctrl_regs(c, r);
    if (finalize_only == 2) c->arrive.v = 0;
}

hipError_t launch_step_ctrl(Ctrl* c, int finalize_only, hipStream_t st)
{
    hipLaunchKernelGGL(step_ctrl_kernel, dim3(1), dim3(64), 0, st, c, finalize_only);
    return hipGetLastError();
}

// Positivity limiter: when the step just run was rejected, copy its input
// state (u^n) over its output buffer, so the retry finds u^n where the next
// step reads its input.  A no-op otherwise.
__global__ __launch_bounds__(256) void restore_kernel(const Ctrl* c, const uint4* src, uint4* dst,
                                                      size_t n16)
{
    if (!c->reject || !c->active || c->done) return;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16;
         i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

hipError_t launch_restore(const Ctrl* c, const void* src, void* dst, size_t bytes, hipStream_t st)
{
    const size_t n16 = bytes / 16;
    size_t g = (n16 + 255) / 256;
    if (g > 2048) g = 2048;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(restore_kernel, dim3((unsigned)g), dim3(256), 0, st, c,
                       static_cast<const uint4*>(src), static_cast<uint4*>(dst), n16);
    return hipGetLastError();
}

// FP64 exchange layout <-> internal view (mixed precision splits mode 0
// into FP64 planes and modes >= 1 into FP32 planes).
template <typename TB>
__global__ __launch_bounds__(256) void convert_kernel(int to_internal, int nmodes, int64_t ncell,
                                                      int64_t total, const double* fp64, double* out64,
                                                      StateView<TB> v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = i % ncell;
        const int64_t rest = i / ncell;
        const int l = (int)(rest % nmodes);
        const int var = (int)(rest / nmodes);
        if (l == 0) {
            double* p = v.m0 + var * v.s0 + c;
            if (to_internal)
                *p = fp64[i];
            else
                out64[i] = *p;
        } else {
            TB* p = v.hi + var * v.sv + (int64_t)(l - 1) * v.sl + c;
            if (to_internal)
                *p = (TB)fp64[i];
            else
                out64[i] = (double)*p;
        }
    }
}

template <typename TB>
hipError_t launch_convert(int to_internal, int nv, int nmodes, int64_t ncell, const double* fp64,
                          StateView<TB> v, hipStream_t st)
{
    const int64_t total = (int64_t)nv * nmodes * ncell;
    int64_t g = (total + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL((convert_kernel<TB>), dim3((unsigned)g), dim3(256), 0, st, to_internal, nmodes,
                       ncell, total, fp64, const_cast<double*>(fp64), v);
    return hipGetLastError();
}

// Deterministic FP64 sum over cells of the cell averages of each variable,
// in two passes with a fixed partition: kLedgerParts workgroups per variable
// each sum one contiguous chunk (fixed strided partial sums, fixed-order LDS
// tree), then one workgroup per variable sums the partials in a fixed-order
// tree.  The result does not depend on scheduling.
template <typename TB>
__global__ __launch_bounds__(256) void ledger_part_kernel(int64_t ncell, StateView<TB> u,
                                                          double* part)
{
    __shared__ double s[256];
    const int var = blockIdx.y;
    const int64_t chunk = (ncell + kLedgerParts - 1) / kLedgerParts;
    const int64_t c0 = (int64_t)blockIdx.x * chunk;
    const int64_t c1 = c0 + chunk < ncell ? c0 + chunk : ncell;
    const double* p = u.m0 + var * u.s0;
    double acc = 0.0;
    for (int64_t c = c0 + threadIdx.x; c < c1; c += 256) acc += p[c];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[var * kLedgerParts + blockIdx.x] = s[0];
}

__global__ __launch_bounds__(kLedgerParts) void ledger_sum_kernel(const double* part, double vol,
                                                                  double* out)
{
    __shared__ double s[kLedgerParts];
    const int var = blockIdx.x;
    s[threadIdx.x] = part[var * kLedgerParts + threadIdx.x];
    __syncthreads();
    for (int w = kLedgerParts / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[var] = vol * s[0];
}

template <typename TB>
hipError_t launch_ledger(int nv, int64_t ncell, StateView<TB> u, double cell_volume, double* out,
                         double* part, hipStream_t st)
{
    hipLaunchKernelGGL((ledger_part_kernel<TB>), dim3(kLedgerParts, nv), dim3(256), 0, st, ncell, u,
                       part);
    hipLaunchKernelGGL(ledger_sum_kernel, dim3(nv), dim3(kLedgerParts), 0, st, part, cell_volume,
                       out);
    return hipGetLastError();
}

// Final-state check (1D Euler): density and pressure in FP64 at every
// Gauss point and both trace points; minima in minvals[0..1] (bit-ordered
// atomicMin over non-negative values; a non-positive value records 0 and
// latches DG_ERR_POSITIVITY, a NaN latches DG_ERR_NONFINITE).
template <int K, typename TB>
__global__ __launch_bounds__(256) void check1d_kernel(StateView<TB> u, int64_t n, PhysParams phys,
                                                      Ctrl* c, unsigned long long* minvals, int pp)
{
    constexpr int Q = K + 1;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double mr = INFINITY, mp = INFINITY;
    if (j < n) {
        double u0[3], uh[3][K > 0 ? K : 1];
        for (int v = 0; v < 3; ++v) {
            u0[v] = u.m0[v * u.s0 + j];
            for (int l = 1; l <= K; ++l) uh[v][l - 1] = (double)u.hi[v * u.sv + (l - 1) * u.sl + j];
        }
        bool bad = false, nonfin = false;
#pragma unroll
        for (int q = 0; q < Q + 2; ++q) {
            double w[3];
            for (int v = 0; v < 3; ++v) {
                double s = u0[v];
                for (int l = 1; l <= K; ++l)
                    s += uh[v][l - 1] * (q < Q ? leg_at(Q, q, l) : q == Q ? dtrace_l(l, 0) : 1.0);
                w[v] = s;
            }
            const double p = Phys1D<EULER>::pressure(w, phys);
            if (!isfinite(w[0]) || !isfinite(p) || !isfinite(w[1])) nonfin = true;
            if (!(w[0] > 0.0) || !(p > 0.0)) bad = true;
            mr = w[0] < mr ? w[0] : mr;
            mp = p < mp ? p : mp;
        }
        // with the positivity limiter, point values sit at its margin up to
        // rounding: only an inadmissible cell average is an error
        if (pp) bad = !(u0[0] > 0.0) || !(Phys1D<EULER>::pressure(u0, phys) > 0.0);
        if (nonfin)
            latch_error(c, -4, j);
        else if (bad)
            latch_error(c, -5, j);
    }
    mr = mr > 0.0 ? mr : 0.0;
    mp = mp > 0.0 ? mp : 0.0;
    // wave minimum
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        double a = __shfl_xor(mr, off, 64), b = __shfl_xor(mp, off, 64);
        mr = a < mr ? a : mr;
        mp = b < mp ? b : mp;
    }
    // workgroup minimum, then one (skippable) atomic per workgroup
    __shared__ double sm[2][4];
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sm[0][wv] = mr;
        sm[1][wv] = mp;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < 4; ++i) {
            mr = sm[0][i] < mr ? sm[0][i] : mr;
            mp = sm[1][i] < mp ? sm[1][i] : mp;
        }
        atomic_min_nonneg(&minvals[0], mr);
        atomic_min_nonneg(&minvals[1], mp);
    }
}

template <typename TB>
hipError_t launch_check1d(int eq, int k, StateView<TB> u, int64_t n, PhysParams phys, Ctrl* c,
                          double* minvals, int pp, hipStream_t st)
{
    if (eq != EULER) return hipSuccess;
    dim3 grid((unsigned)((n + 255) / 256)), block(256);
    unsigned long long* mv = reinterpret_cast<unsigned long long*>(minvals);
    switch (k) {
    case 0: hipLaunchKernelGGL((check1d_kernel<0, TB>), grid, block, 0, st, u, n, phys, c, mv, pp); break;
    case 1: hipLaunchKernelGGL((check1d_kernel<1, TB>), grid, block, 0, st, u, n, phys, c, mv, pp); break;
    case 2: hipLaunchKernelGGL((check1d_kernel<2, TB>), grid, block, 0, st, u, n, phys, c, mv, pp); break;
    default: hipLaunchKernelGGL((check1d_kernel<3, TB>), grid, block, 0, st, u, n, phys, c, mv, pp); break;
    }
    return hipGetLastError();
}

#define DG_INST(TB)                                                                                \
    template hipError_t launch_convert<TB>(int, int, int, int64_t, const double*, StateView<TB>,   \
                                           hipStream_t);                                           \
    template hipError_t launch_ledger<TB>(int, int64_t, StateView<TB>, double, double*, double*,  \
                                          hipStream_t);                                           \
    template hipError_t launch_check1d<TB>(int, int, StateView<TB>, int64_t, PhysParams, Ctrl*,    \
                                           double*, int, hipStream_t);
DG_INST(double)
DG_INST(float)
#undef DG_INST

}  // namespace dg
