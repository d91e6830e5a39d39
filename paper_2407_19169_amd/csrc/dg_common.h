// dg_common.h — device-side building blocks shared by the 1D, 2D and batched
// kernels of the RKDG + jump-filter library (gfx950).
//
// Basis: standard Legendre polynomials P_l on [-1, 1], P_0 = 1, so the mode-0
// coefficient is the cell average (arXiv:2407.19169, Sec. 2.1).  Tables are
// compile-time constants built from the closed forms of P_0..P_3, their
// derivatives and the Gauss-Legendre rules with 1..4 points, so every loop
// over modes or quadrature points folds to straight-line FMA code.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dg_tables.h"

namespace dg {

constexpr int kMaxDeg = 3;

enum Eq { ADV = 0, BURGERS = 1, EULER = 2 };
enum Bc { BC_PERIODIC = 0, BC_OUTFLOW = 1, BC_REFLECT = 2, BC_DIRICHLET = 3, BC_DMR_WALL = 4,
          BC_DMR_TOP = 5 };
enum Filter { F_NONE = 0, F_JUMP = 1, F_HYBRID = 2 };

// ---------------------------------------------------------------- basis --
// Gauss-Legendre nodes/weights (Q = 1..4, ascending nodes) and P_l, P_l'
// at the nodes: correctly rounded constants from dg_tables.h.
__host__ __device__ constexpr double gl_node(int Q, int i) { return kGaussX[Q - 1][i]; }
__host__ __device__ constexpr double gl_weight(int Q, int i) { return kGaussW[Q - 1][i]; }
__host__ __device__ constexpr double leg_at(int Q, int i, int l) { return kLegAt[Q - 1][i][l]; }
__host__ __device__ constexpr double dleg_at(int Q, int i, int l) { return kDLegAt[Q - 1][i][l]; }
// d^m/dx^m P_l at x = +1: (l+m)! / (2^m m! (l-m)!), zero for m > l.
__host__ __device__ constexpr double dtrace_r(int l, int m)
{
    return m > l ? 0.0
         : m == 0 ? 1.0
         : l == 1 ? 1.0
         : l == 2 ? 3.0
         : (m == 1 ? 6.0 : 15.0);
}
// ... at x = -1: (-1)^(l+m) times the value at +1.
__host__ __device__ constexpr double dtrace_l(int l, int m)
{
    return ((l + m) & 1) ? -dtrace_r(l, m) : dtrace_r(l, m);
}
// Weight of the reference-coordinate derivative jump of order m in the
// damping sum: m(m+1) h^m |[d^m u/dx^m]| = m(m+1) 2^m |[d^m u/dxi^m]|.
__host__ __device__ constexpr double jump_weight(int m)
{
    return m == 0 ? 1.0 : (double)(m * (m + 1)) * (double)(1 << m);
}

// ------------------------------------------------------------- physics --
struct PhysParams {
    double gamma;
    double a[2];   // advection velocity
    int flux;      // numerical flux (Euler): FLUX_LLF, FLUX_HLL, FLUX_HLLC
};

// Numerical fluxes: Sec. 3 computes with the local Lax-Friedrichs flux and
// names HLL and HLLC as alternatives that work with the filter as well.
enum { FLUX_LLF = 0, FLUX_HLL = 1, FLUX_HLLC = 2 };

// Square root for the wave speeds.  FP64: for x in [2^-1000, 2^1000],
// Markstein's iteration from the hardware reciprocal square root estimate y:
// g = x y, h = y/2, one coupled Newton step (r = 1/2 - g h, g <- g + g r,
// h <- h + h r), then two corrections g <- g + (x - g^2) h; this is the
// library's own sequence without its rescaling of extreme arguments, which
// takes the other values (zero, negative, non-finite, extreme) here.  FP32:
// the hardware square root (1 ulp; the correctly rounded FP32 root takes ten
// instructions).
template <typename T>
__device__ __forceinline__ T tsqrt(T x)
{
    if (!(x >= 0x1p-1000 && x <= 0x1p1000)) return sqrt(x);
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    const double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    g = fma(fma(-g, g, x), h, g);
    return fma(fma(-g, g, x), h, g);
}
template <>
__device__ __forceinline__ float tsqrt<float>(float x) { return __builtin_amdgcn_sqrtf(x); }

// 1/x for the flux arithmetic (the reciprocal of a density): FP64 by two
// Newton-Raphson steps r <- r + r (1 - x r) from the hardware estimate,
// within about an ulp of the rounded quotient for normal x (5 instructions
// where the IEEE quotient takes 10); FP32 the hardware reciprocal (1 ulp).
// A zero or non-finite x gives a non-finite result, as the quotient does.
template <typename T>
__device__ __forceinline__ T trcp(T x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
template <>
__device__ __forceinline__ float trcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }

template <int EQ>
struct Phys1D;

template <>
struct Phys1D<ADV> {
    static constexpr int NV = 1;
    template <typename T>
    __device__ static void flux(const T* u, T* f, const PhysParams& p) { f[0] = (T)p.a[0] * u[0]; }
    template <typename T>
    __device__ static T speed(const T* u, const PhysParams& p) { return fabs((T)p.a[0]); }
    template <typename T>
    __device__ static T enthalpy(const T* u, const PhysParams& p) { return (T)1; }
    template <typename T>
    __device__ static T flux_speed(const T* u, T* f, const PhysParams& p, T* pr_out = nullptr)
    {
        flux(u, f, p);
        if (pr_out) *pr_out = (T)1;
        return speed(u, p);
    }
    template <typename T>
    __device__ static T flux_pressure(const T* u, T* f, const PhysParams& p)
    {
        flux(u, f, p);
        return (T)1;
    }
};

template <>
struct Phys1D<BURGERS> {
    static constexpr int NV = 1;
    template <typename T>
    __device__ static void flux(const T* u, T* f, const PhysParams& p) { f[0] = (T)0.5 * u[0] * u[0]; }
    template <typename T>
    __device__ static T speed(const T* u, const PhysParams& p) { return fabs(u[0]); }
    template <typename T>
    __device__ static T enthalpy(const T* u, const PhysParams& p) { return (T)1; }
    template <typename T>
    __device__ static T flux_speed(const T* u, T* f, const PhysParams& p, T* pr_out = nullptr)
    {
        flux(u, f, p);
        if (pr_out) *pr_out = (T)1;
        return speed(u, p);
    }
    template <typename T>
    __device__ static T flux_pressure(const T* u, T* f, const PhysParams& p)
    {
        flux(u, f, p);
        return (T)1;
    }
};

template <>
struct Phys1D<EULER> {
    static constexpr int NV = 3;
    template <typename T>
    __device__ static T pressure(const T* u, const PhysParams& p)
    {
        return ((T)p.gamma - (T)1) * (u[2] - (T)0.5 * u[1] * (u[1] * trcp<T>(u[0])));
    }
    template <typename T>
    __device__ static void flux(const T* u, T* f, const PhysParams& p)
    {
        T vel = u[1] / u[0];
        T pr = ((T)p.gamma - (T)1) * (u[2] - (T)0.5 * u[1] * vel);
        f[0] = u[1];
        f[1] = u[1] * vel + pr;
        f[2] = vel * (u[2] + pr);
    }
    // (speed and enthalpy from one reciprocal of the density, trcp)
    template <typename T>
    __device__ static T speed(const T* u, const PhysParams& p)
    {
        const T ir = trcp<T>(u[0]);
        const T vel = u[1] * ir;
        const T pr = ((T)p.gamma - (T)1) * (u[2] - (T)0.5 * u[1] * vel);
        return fabs(vel) + tsqrt<T>((T)p.gamma * pr * ir);
    }
    template <typename T>
    __device__ static T enthalpy(const T* u, const PhysParams& p)
    {
        const T ir = trcp<T>(u[0]);
        const T pr = ((T)p.gamma - (T)1) * (u[2] - (T)0.5 * u[1] * (u[1] * ir));
        return (u[2] + pr) * ir;
    }
    // flux and speed of one state (an interface flux's side) from one
    // reciprocal of the density; the pressure is returned in *pr_out
    template <typename T>
    __device__ static T flux_speed(const T* u, T* f, const PhysParams& p, T* pr_out = nullptr)
    {
        const T ir = trcp<T>(u[0]);
        const T vel = u[1] * ir;
        const T pr = ((T)p.gamma - (T)1) * (u[2] - (T)0.5 * u[1] * vel);
        f[0] = u[1];
        f[1] = u[1] * vel + pr;
        f[2] = vel * (u[2] + pr);
        if (pr_out) *pr_out = pr;
        return fabs(vel) + tsqrt<T>((T)p.gamma * pr * ir);
    }
    // flux of one state, returning the pressure it used
    template <typename T>
    __device__ static T flux_pressure(const T* u, T* f, const PhysParams& p)
    {
        const T vel = u[1] * trcp<T>(u[0]);
        const T pr = ((T)p.gamma - (T)1) * (u[2] - (T)0.5 * u[1] * vel);
        f[0] = u[1];
        f[1] = u[1] * vel + pr;
        f[2] = vel * (u[2] + pr);
        return pr;
    }
};

// HLL and HLLC fluxes of the Euler equations across a face (Harten, Lax
// and van Leer; Toro, Spruce and Speares), from the two states, their
// physical fluxes fl, fr and pressures.  1D (NV = 3): the normal momentum
// is component 1; 2D (NV = 4): component 1 (x faces) or 2 (ydir), the
// other momentum being tangential.  Wave speeds are Davis's estimates
// S_L = min(u_L - c_L, u_R - c_R), S_R = max(u_L + c_L, u_R + c_R).  HLL:
//   (S_R f_L - S_L f_R + S_L S_R (U_R - U_L)) / (S_R - S_L) for S_L < 0 < S_R;
// HLLC: the contact speed
//   S* = (p_R - p_L + m_L (S_L - u_L) - m_R (S_R - u_R)) / (rho_L (S_L - u_L) - rho_R (S_R - u_R)),
// and on the side K that holds the face f_K + S_K (U*_K - U_K) with
//   U*_K = rho_K (S_K - u_K) / (S_K - S*) (1, S* [normal], v_K [tangential],
//          E_K / rho_K + (S* - u_K) (S* + p_K / (rho_K (S_K - u_K)))).
// Outside the fan the upwind flux is taken.  (Selects only: the face
// direction may be a run-time value.)
template <int NV, typename T>
__device__ __forceinline__ void hll_euler(int kind, bool ydir, const T* ul, const T* ur, const T* fl,
                                          const T* fr, T pl, T pr, T gamma, T* fh)
{
    const bool y = NV == 4 && ydir;
    const T mL = y ? ul[2] : ul[1], mR = y ? ur[2] : ur[1];
    const T uL = mL / ul[0], uR = mR / ur[0];
    const T cL = tsqrt<T>(gamma * pl / ul[0]), cR = tsqrt<T>(gamma * pr / ur[0]);
    // fmin / fmax: a sound speed that is NaN (a state with negative
    // pressure) leaves the bound to the other state
    const T sL = fmin(uL - cL, uR - cR);
    const T sR = fmax(uL + cL, uR + cR);
    if (!(sL < (T)0)) {
#pragma unroll
        for (int v = 0; v < NV; ++v) fh[v] = fl[v];
        return;
    }
    if (!(sR > (T)0)) {
#pragma unroll
        for (int v = 0; v < NV; ++v) fh[v] = fr[v];
        return;
    }
    if (kind == FLUX_HLL) {
        const T inv = (T)1 / (sR - sL);
#pragma unroll
        for (int v = 0; v < NV; ++v) fh[v] = (sR * fl[v] - sL * fr[v] + sL * sR * (ur[v] - ul[v])) * inv;
        return;
    }
    const T dL = ul[0] * (sL - uL), dR = ur[0] * (sR - uR);
    const T sS = (pr - pl + mL * (sL - uL) - mR * (sR - uR)) / (dL - dR);
    const bool left = !(sS < (T)0);
    T uK[NV], fK[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        uK[v] = left ? ul[v] : ur[v];
        fK[v] = left ? fl[v] : fr[v];
    }
    const T sK = left ? sL : sR, unK = left ? uL : uR, pK = left ? pl : pr, dK = left ? dL : dR;
    const T fac = dK / (sK - sS);
    T us[NV];
    us[0] = fac;
    if constexpr (NV == 4) {
        const T vt = (y ? uK[1] : uK[2]) / uK[0];
        us[1] = y ? fac * vt : fac * sS;
        us[2] = y ? fac * sS : fac * vt;
    } else {
        us[1] = fac * sS;
    }
    us[NV - 1] = fac * (uK[NV - 1] / uK[0] + (sS - unK) * (sS + pK / dK));
#pragma unroll
    for (int v = 0; v < NV; ++v) fh[v] = fK[v] + sK * (us[v] - uK[v]);
}

// Interface flux.  Local Lax-Friedrichs (the default):
// 1/2 (f(a) + f(b)) - 1/2 max(|f'(a)|, |f'(b)|) (b - a); Euler kernels
// compiled with HLLX take HLL or HLLC (p.flux) instead.  (A run-time choice
// in the default kernels would cost them registers.)
template <int EQ, typename T, bool HLLX = false>
__device__ __forceinline__ void llf1d(const T* ul, const T* ur, T* fh, const PhysParams& p,
                                      T* pl = nullptr, T* pr = nullptr)
{
    constexpr int NV = Phys1D<EQ>::NV;
    T fl[NV], fr[NV];
    T pl_ = (T)0, pr_ = (T)0;
    const T al = Phys1D<EQ>::flux_speed(ul, fl, p, &pl_);
    const T ar = Phys1D<EQ>::flux_speed(ur, fr, p, &pr_);
    if (pl) *pl = pl_;
    if (pr) *pr = pr_;
    if constexpr (EQ == EULER && HLLX) {
        hll_euler<NV, T>(p.flux, false, ul, ur, fl, fr, pl_, pr_, (T)p.gamma, fh);
        return;
    }
    T alpha = al > ar ? al : ar;
#pragma unroll
    for (int v = 0; v < NV; ++v) fh[v] = (T)0.5 * (fl[v] + fr[v]) - (T)0.5 * alpha * (ur[v] - ul[v]);
}

// ---------------------------------------------------------- state views --
// Mode 0 always lives in FP64 planes; modes >= 1 live in TB planes
// (TB = double for DG_PREC_FP64, float for DG_PREC_MIXED).  For the FP64
// layout (u[(var*(k+1)+l)*n + j]) hi points at mode 1 of var 0 and shares
// the var stride with m0.
template <typename TB>
struct StateView {
    double* m0;           // mode 0, var v at m0 + v*s0
    TB* hi;               // mode l >= 1, var v at hi + v*sv + (l-1)*sl
    int64_t s0, sv, sl;
};

// ------------------------------------------------------- control block --
// Device-resident run state, in the workspace.  Written by the kernels and
// read back by the host only for reports.
struct Ctrl {
    double t;                        // time at the start of the current step
    double dt;                       // current step
    double t_end;
    double dt_min, dt_max;
    double cfl_num;                  // 1D: cfl*h (dt = cfl_num/alpha); 2D: cfl
    int active;                      // a scheduled step waits to be finalised
    long long steps;
    long long max_steps;             // absolute step limit of the current run
    long long troubled;              // hybrid: troubled cells summed over stages
    int last;                        // the scheduled step ends exactly at t_end
    int done;                        // no further step will run
    int status;                      // first error code latched (dg_status)
    int reject;                      // positivity limiter: a stage left a bad cell average
    long long first_bad;             // cell index of that error
    double bflux[4];                 // boundary-flux ledger (FP64)
    double bstage[3][8];             // per-stage boundary fluxes: lo[4], hi[4]
    long long restarts;              // steps retried with half dt (positivity limiter)
    int retries;                     // consecutive retries of the current step
    int pad;
    // Accumulators the stage kernels update with atomics, on lines apart
    // from the fields above (read as each kernel starts).  Each stage's eta
    // maximum has a 128-byte line of its own: a stage reads the previous
    // stage's maximum while its own workgroups accumulate into theirs, and
    // loads of a line that atomics are updating measured slower.
    alignas(128) unsigned long long alpha_bits;  // CFL max (atomicMax of a non-negative double)
    unsigned long long exp_bits;                 // largest damping exponent seen
    unsigned int tcount[3];                      // hybrid: troubled-list entries per stage
    struct alignas(128) Line {
        unsigned long long v;
    } eta_line[3];                               // hybrid: max eta per stage (.v)
    Line arrive;                                 // workgroups of a launch that have finished
    Line pcount;                                 // 2D positivity limiter: cells listed this stage (.v)
};

// Retries of one step with halved dt (positivity limiter) before a run stops.
constexpr int kMaxRetries = 40;

// atomicMax/atomicMin over doubles through their bit patterns; valid for
// non-negative values (IEEE-754 order equals unsigned order there) and
// propagates NaN (its bit pattern exceeds every finite one).
// The atomic is issued only when v exceeds the value already there (read
// from L2, coherent across the device): thousands of workgroups reducing
// into one address otherwise serialise on it.  Within a reduction the
// stored value only grows, so a skipped update can never lose the maximum.
__device__ __forceinline__ void atomic_max_nonneg(unsigned long long* p, double v)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    if (b > __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(p, b);
}

// The minimum counterpart (the stored value only falls within a reduction).
__device__ __forceinline__ void atomic_min_nonneg(unsigned long long* p, double v)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    if (b < __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMin(p, b);
}

// Wavefront (64 lanes) maximum.
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        double o = __shfl_xor(v, off, 64);
        v = (o > v || o != o) ? o : v;
    }
    return v;
}

// A double stored with an agent-scope atomic store (visible at the point of
// coherence without a cache write-back).
__device__ __forceinline__ void store_coherent(double* p, double v)
{
    __hip_atomic_store(reinterpret_cast<long long*>(p), __double_as_longlong(v), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void latch_error(Ctrl* c, int code, long long cell)
{
    // (an atomic store: the step control may run in a workgroup of the same
    // launch, which reads the cell at the point of coherence)
    if (atomicCAS(&c->status, 0, code) == 0)
        __hip_atomic_store(&c->first_bad, cell, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace dg

namespace dg {
// e^x for the filter factors: FP64 the library exponential; FP32 the
// hardware base-2 exponential of x log2(e) (a few ulp where the factor is
// not negligible, against about ten instructions for the library's).
template <typename T>
__device__ __forceinline__ T texp(T x) { return exp(x); }
template <>
__device__ __forceinline__ float texp<float>(float x) { return __builtin_amdgcn_exp2f(x * 0x1.715476p+0f); }
}  // namespace dg
