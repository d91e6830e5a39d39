// dg1d.hip — 1D RKDG stage, jump filter, hybrid limiter and CFL kernels
// for gfx950 (arXiv:2407.19169, Sec. 2.1, 2.4, Sec. 3 and Algorithm 1).
//
// Mapping: one thread per cell; the stage kernel runs 256-thread workgroups
// (4 wave64) on large grids and single-wavefront tiles on small ones, the
// other kernels 256-thread workgroups.  State lives in
// structure-of-arrays planes so every load/store of a mode plane is one
// coalesced 64-lane access.  A workgroup stages its cells' interface traces
// in LDS, so each interface flux is evaluated once per tile.  The fused
// kernel carries a 2-cell halo: it recomputes the unfiltered stage output of
// one neighbour on each side so that the jump filter (which needs the
// post-update traces of both neighbours) runs in the same pass, and the
// stage costs one read of u^(s) (+ u^n) and one write.
#include "dg_kernels.h"

namespace dg {

namespace {

template <int K, int NV, typename TB>
__device__ __forceinline__ void load_cell(const StateView<TB>& s, int64_t c, double (&u0)[NV],
                                          TB (&uh)[NV][K > 0 ? K : 1])
{
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        u0[v] = s.m0[v * s.s0 + c];
#pragma unroll
        for (int l = 1; l <= K; ++l) uh[v][l - 1] = s.hi[v * s.sv + (l - 1) * s.sl + c];
    }
}

template <int K, int NV, typename TB>
__device__ __forceinline__ void store_cell(const StateView<TB>& s, int64_t c, const double (&u0)[NV],
                                           const TB (&uh)[NV][K > 0 ? K : 1])
{
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        s.m0[v * s.s0 + c] = u0[v];
#pragma unroll
        for (int l = 1; l <= K; ++l) s.hi[v * s.sv + (l - 1) * s.sl + c] = uh[v][l - 1];
    }
}

__device__ __forceinline__ int64_t wrap(int64_t c, int64_t n)
{
    int64_t r = c % n;
    return r < 0 ? r + n : r;
}

// Ghost value outside a domain end for the flux (m = 0 only).
template <int NV, typename T>
__device__ __forceinline__ void ghost_state(int bc, const double* dir, const T* inner, T* g)
{
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        if (bc == BC_REFLECT)
            g[v] = (v == 1) ? -inner[v] : inner[v];
        else if (bc == BC_DIRICHLET)
            g[v] = (T)dir[v];
        else
            g[v] = inner[v];
    }
}

// |ghost - inner| of the m-th derivative outside a domain end (jump filter).
template <typename T>
__device__ __forceinline__ T ghost_jump(int bc, int m, int v, double dirv, T inner)
{
    if (bc == BC_REFLECT) {
        bool odd = ((m & 1) != 0) != (v == 1);   // ghost = -inner
        return odd ? (T)2 * fabs(inner) : (T)0;
    }
    if (bc == BC_DIRICHLET) return m == 0 ? fabs((T)dirv - inner) : fabs(inner);
    return (T)0;  // outflow: ghost derivatives equal the interior ones
}

// Shu-Osher combination of stage `stage` (SSP-RK3).
__device__ __forceinline__ double combine(int stage, double un, double adv)
{
    return stage == 0 ? adv : stage == 1 ? 0.75 * un + 0.25 * adv : (1.0 / 3.0) * un + (2.0 / 3.0) * adv;
}
template <typename T>
__device__ __forceinline__ T combine_t(int stage, T un, T adv)
{
    return stage == 0 ? adv
         : stage == 1 ? (T)0.75 * un + (T)0.25 * adv
                      : (T)(1.0 / 3.0) * un + (T)(2.0 / 3.0) * adv;
}

// Hybrid pass B applied on load (deferred blend): a cell whose eta exceeds 1
// gets u^l <- [omega + (1 - omega) exp(-E^l)] u^l, omega = (M - eta)/(M - 1),
// with the same operations as the pass-B kernel applies to memory.
// What one cell's blend reads: eta, the exponents and the stage maximum M
// (read whether or not the cell is troubled, with the cell's state).
template <int K, typename TB>
struct BlendIn {
    double eta, M;
    TB e[K > 0 ? K : 1];
};

template <int K, typename TB, typename D>
__device__ __forceinline__ BlendIn<K, TB> blend_fetch(const D& bl, int64_t n, int64_t c)
{
    BlendIn<K, TB> b;
    b.eta = (double)bl.eta[c];
#pragma unroll
    for (int l = 1; l <= K; ++l) b.e[l - 1] = bl.E[(int64_t)(l - 1) * n + c];
    b.M = __longlong_as_double((long long)*bl.M);
    return b;
}

// An empty asm statement that uses the fetched values: the compiler cannot
// sink their loads into the troubled-cell branch, so they travel with the
// state loads instead of costing troubled cells a second trip to memory.
template <int K, typename TB>
__device__ __forceinline__ void blend_pin(const BlendIn<K, TB>& b)
{
    asm volatile("" ::"v"(b.eta), "s"(b.M));
#pragma unroll
    for (int l = 0; l < K; ++l) asm volatile("" ::"v"(b.e[l]));
}

template <int K, int NV, typename TB>
__device__ __forceinline__ void blend_apply(const BlendIn<K, TB>& b, TB (&uh)[NV][K > 0 ? K : 1])
{
    if constexpr (K > 0) {
        if (!(b.eta > 1.0)) return;
        const double w = (b.M - b.eta) / (b.M - 1.0);
#pragma unroll
        for (int l = 1; l <= K; ++l) {
            const TB f = (TB)(w + (1.0 - w) * exp(-(double)b.e[l - 1]));
#pragma unroll
            for (int v = 0; v < NV; ++v) uh[v][l - 1] *= f;
        }
    }
}

// ------------------------------------------------ positivity limiter --
// Zhang and Shu's positivity-preserving limiter for the Euler equations,
// applied after the filter (the paper's Sec. 3.2 examples with extreme
// positivity demands).  Test points of a cell: the N-point Gauss-Lobatto
// nodes, N = ceil((k+3)/2) (both ends, and the centre for N = 3), followed
// by the K+1 Gauss points of the volume rule.
template <int K>
struct PPPoints {
    static constexpr int N = (K + 4) / 2;
    static constexpr int NP = (N == 3 ? 3 : 2) + K + 1;
};

// P_l at test point i.
template <int K>
__device__ __forceinline__ constexpr double pp_leg(int i, int l)
{
    constexpr int N = PPPoints<K>::N;
    return i == 0 ? ((l & 1) ? -1.0 : 1.0)
         : i == 1 ? 1.0
         : (N == 3 && i == 2) ? (l == 0 ? 1.0 : l == 2 ? -0.5 : 0.0)
         : leg_at(K + 1, i - (N == 3 ? 3 : 2), l);
}

template <int K, typename TB>
__device__ __forceinline__ void pp_point(const double (&u0)[3], const TB (&uh)[3][K > 0 ? K : 1],
                                         int i, double (&w)[3])
{
#pragma unroll
    for (int v = 0; v < 3; ++v) {
        double s = u0[v];
#pragma unroll
        for (int l = 1; l <= K; ++l) s += (double)uh[v][l - 1] * pp_leg<K>(i, l);
        w[v] = s;
    }
}

// Point value and the sums of the magnitudes of its terms.
template <int K, typename TB>
__device__ __forceinline__ void pp_point_abs(const double (&u0)[3], const TB (&uh)[3][K > 0 ? K : 1],
                                             int i, double (&w)[3], double (&wa)[3])
{
#pragma unroll
    for (int v = 0; v < 3; ++v) {
        double s = u0[v], sa = fabs(u0[v]);
#pragma unroll
        for (int l = 1; l <= K; ++l) {
            const double t = (double)uh[v][l - 1] * pp_leg<K>(i, l);
            s += t;
            sa += fabs(t);
        }
        w[v] = s;
        wa[v] = sa;
    }
}

__device__ __forceinline__ double pp_pressure(double gamma, const double (&w)[3])
{
    return (gamma - 1.0) * (w[2] - 0.5 * w[1] * w[1] / w[0]);
}

// Rounding margin of the pressure at a point (8 units of roundoff of the
// arithmetic the fluxes use, times the magnitudes that cancel in
// E - m^2 / (2 rho)): below it the point pressure has no reliable sign.
template <typename TB>
__device__ __forceinline__ double pp_margin(const double (&w)[3], const double (&wa)[3])
{
    constexpr double ur = sizeof(TB) == 4 ? 0x1p-23 : 0x1p-52;
    const double kin = 0.5 * w[1] * w[1] / w[0];
    return 8.0 * ur * (wa[2] + fabs(w[1]) * wa[1] / w[0] + kin * wa[0] / w[0]);
}

// True when the limiter provably leaves the cell unchanged: since |P_l| <= 1
// on [-1, 1], rho_bar - sum_l |rho_l| bounds the density and
// (gamma - 1) (E_lo - M_hi^2 / (2 rho_lo)) the pressure from below at every
// point of the cell; both exceed twice the largest threshold and rounding
// margin the limiter could apply there (the margins' 8 units of roundoff
// also cover the rounding of the point values and of the verification in
// the modes' precision), so no test point is limited and the verification
// passes at once.
template <int K, typename TB>
__device__ __forceinline__ bool pp_clear(const double (&u0)[3], const TB (&uh)[3][K > 0 ? K : 1],
                                         double gamma)
{
    constexpr double ur = sizeof(TB) == 4 ? 0x1p-23 : 0x1p-52;
    double sa[3];
#pragma unroll
    for (int v = 0; v < 3; ++v) {
        double t = 0.0;
#pragma unroll
        for (int l = 0; l < K; ++l) t += fabs((double)uh[v][l]);
        sa[v] = t;
    }
    const double rlo = u0[0] - sa[0], sr = fabs(u0[0]) + sa[0];
    if (!(rlo > 2.0 * (1e-13 + 8.0 * ur * sr))) return false;
    const double mhi = fabs(u0[1]) + sa[1];
    const double elo = u0[2] - sa[2], se = fabs(u0[2]) + sa[2];
    // (1/rlo by the reciprocal helper: the margins below are two-fold)
    const double irlo = trcp<double>(rlo);
    const double kin = 0.5 * mhi * mhi * irlo;
    const double plo = (gamma - 1.0) * (elo - kin);
    const double mmax = 8.0 * ur * (se + 2.0 * kin + kin * sr * irlo);
    return plo > 2.0 * (1e-13 + mmax);
}

// Limit one cell in place: scale the density's modes >= 1 so the density
// at every test point is >= eps_r, then all modes >= 1 so the pressure is
// >= eps_p (largest admissible t in [0, 1] on the segment from the average
// to each point value, by 60 bisection steps; the pressure is concave
// along it).  FP64 modes: eps = min(1e-13, rho_bar, p_bar) as in Zhang and
// Shu, raised to the rounding margins of the point values (8 u sum |rho_l
// P_l| for the density, pp_margin for the pressure), which vanish in exact
// arithmetic.  FP32 modes (mixed precision): the margins use FP32's unit
// roundoff, which also covers rounding the limited modes to FP32.  The
// average is never changed; an inadmissible average is left for the
// caller's check.
template <int K, typename TB>
__device__ __forceinline__ void pp_limit(double (&u0)[3], TB (&uh)[3][K > 0 ? K : 1], double gamma)
{
    if constexpr (K > 0) {
        if (pp_clear<K, TB>(u0, uh, gamma)) return;
        constexpr int NP = PPPoints<K>::NP;
        constexpr bool kFP32 = sizeof(TB) == 4;
        const double pb = pp_pressure(gamma, u0);
        if (!(u0[0] > 0.0) || !(pb > 0.0)) return;
        double eps = 1e-13;
        if (u0[0] < eps) eps = u0[0];
        if (pb < eps) eps = pb;
        double eps_r = eps;
        const double eps_p = eps;
        constexpr double ur = kFP32 ? 0x1p-23 : 0x1p-52;
        double rmin = INFINITY;
        for (int i = 0; i < NP; ++i) {
            double w[3], wa[3];
            pp_point_abs<K, TB>(u0, uh, i, w, wa);
            if (w[0] < rmin) rmin = w[0];
            const double m = 8.0 * ur * wa[0];
            if (m > eps_r) eps_r = m;
        }
        if (eps_r > u0[0]) eps_r = u0[0];
        if (rmin < eps_r) {
            double th = (u0[0] - eps_r) / (u0[0] - rmin);
            if (th < 0.0) th = 0.0;
#pragma unroll
            for (int l = 0; l < K; ++l) uh[0][l] = (TB)((double)uh[0][l] * th);
        }
        double theta = 1.0;
        for (int i = 0; i < NP; ++i) {
            double w[3], wa[3];
            pp_point_abs<K, TB>(u0, uh, i, w, wa);
            double eps_i = eps_p;
            if (w[0] > 0.0) {
                const double m = pp_margin<TB>(w, wa);
                if (m > eps_i) eps_i = m;
            }
            if (eps_i > pb) eps_i = pb;
            if (pp_pressure(gamma, w) >= eps_i) continue;
            double lo = 0.0, hi = 1.0;
            for (int it = 0; it < 60; ++it) {
                const double mid = 0.5 * (lo + hi);
                double wm[3];
#pragma unroll
                for (int v = 0; v < 3; ++v) wm[v] = u0[v] + mid * (w[v] - u0[v]);
                if (pp_pressure(gamma, wm) >= eps_i)
                    lo = mid;
                else
                    hi = mid;
            }
            if (lo < theta) theta = lo;
        }
        if (theta < 1.0) {
#pragma unroll
            for (int v = 0; v < 3; ++v)
#pragma unroll
                for (int l = 0; l < K; ++l) uh[v][l] = (TB)((double)uh[v][l] * theta);
        }
        // Positivity in the fluxes' own arithmetic (precision TB, pressure
        // as the flux computes it): near vacuum the point values of the
        // scaled coefficients can differ in sign from the segment values
        // by rounding, so the modes >= 1 are halved until every test point
        // is positive (dropped after 50 halvings).
        for (int halving = 0; halving <= 50; ++halving) {
            bool ok = true;
            for (int i = 0; i < NP && ok; ++i) {
                TB w[3];
#pragma unroll
                for (int v = 0; v < 3; ++v) {
                    TB s = (TB)u0[v];
#pragma unroll
                    for (int l = 1; l <= K; ++l) s += uh[v][l - 1] * (TB)pp_leg<K>(i, l);
                    w[v] = s;
                }
                const TB vel = w[1] / w[0];
                const TB pr = ((TB)gamma - (TB)1) * (w[2] - (TB)0.5 * w[1] * vel);
                ok = w[0] > (TB)0 && pr > (TB)0;
            }
            if (ok) break;
            const TB f = halving < 50 ? (TB)0.5 : (TB)0;
#pragma unroll
            for (int v = 0; v < 3; ++v)
#pragma unroll
                for (int l = 0; l < K; ++l) uh[v][l] *= f;
        }
    }
}

__device__ __forceinline__ bool pp_admissible(const double (&u0)[3], double gamma)
{
    return u0[0] > 0.0 && pp_pressure(gamma, u0) > 0.0;
}

// Limiter (Euler with the limiter on) + average check of one own output
// cell; returns the CFL quantity of its average.
template <int EQ, int K, typename TB, int NV>
__device__ __forceinline__ double finish_cell(const Args1D<TB>& a, int64_t c, double (&v0)[NV],
                                              TB (&vh)[NV][K > 0 ? K : 1], bool limit)
{
    if constexpr (EQ == EULER) {
        if (a.pp && limit) {
            pp_limit<K, TB>(v0, vh, a.phys.gamma);
            if (!pp_admissible(v0, a.phys.gamma) && a.reject) atomicOr(a.reject, 1);
        }
    }
    // the CFL quantity is only reduced after the last stage of a step
    return (a.alpha_acc || a.want_lam) ? (double)Phys1D<EQ>::speed(v0, a.phys) : 0.0;
}

// Positivity and finiteness of the two states of an interface flux (the
// pressures are those the flux computed).  With the positivity limiter the
// traces sit at its margin up to rounding: only non-finite values latch.
template <typename TB, typename T>
__device__ __forceinline__ void trace_check(const Args1D<TB>& a, const T* ul, const T* ur, T pl, T pr,
                                            int64_t cell)
{
    if (!(ul[0] > (T)0) || !(ur[0] > (T)0) || !(pl > (T)0) || !(pr > (T)0)) {
        const bool fin = isfinite((double)ul[0]) && isfinite((double)ur[0]) && isfinite((double)pl) &&
                         isfinite((double)pr);
        if (!fin || !a.pp) latch_error(a.ctrl, fin ? -5 : -4, cell);
    }
}

}  // namespace

// -------------------------------------------------------------------------
// Stage kernel.
//   MODE 0: unfiltered stage output (halo 1)              -> a.out
//   MODE 1: stage + jump filter (halo 2)                  -> a.out
//   MODE 2: stage + hybrid pass A (halo 2): writes the unfiltered output,
//           the jump indicator max and the troubled-cell list (cell, eta,
//           exponents) for pass B.
// With a.alpha != 0 the kernel also accumulates max |f'(u-bar)| of its
// output into ctrl->alpha_bits (the next step's CFL reduction).
// -------------------------------------------------------------------------
template <int EQ, int K, typename TB, int MODE, int BS = 256>
struct Stage1DLds {
    static constexpr int NV = Phys1D<EQ>::NV;
    // phase 1 (traces, fluxes) and phase 2 (mode 0, right derivative
    // traces, later the left-interface jumps) alias
    static constexpr int PH1 = 2 * NV * BS * (int)sizeof(TB);
    static constexpr int PH2 = NV * BS * 8 + (K + 1) * NV * BS * (int)sizeof(TB);
    static constexpr int bytes = MODE == 0 ? PH1 : (PH1 > PH2 ? PH1 : PH2);
};

// One BS-cell tile (tile index blk) of the stage; `lds` provides
// Stage1DLds::bytes of shared memory.  Returns, per thread, the CFL
// quantity of its output cell (*lam_out, 0 for halo / outside lanes) and
// its hybrid indicator (*eta_out); reductions are left to the caller.
template <int EQ, int K, typename TB, int MODE, int BS = 256, bool HLLX = false, int NST = 1>
__device__ __forceinline__ void stage1d_tile(const Args1D<TB>& a, int64_t blk, double dt,
                                             unsigned char* lds, double* lam_out, double* eta_out)
{
    using P = Phys1D<EQ>;
    using T = TB;
    constexpr int NV = P::NV;
    constexpr int K1 = K + 1;
    constexpr int KH = K > 0 ? K : 1;
    // NST = 3: the whole SSP-RK3 step (MODE 0 or 1) in one pass; each stage
    // consumes H1 lanes of halo on each side (the flux, and the filter's
    // neighbour traces)
    static_assert(NST == 1 || (NST == 3 && MODE != 2), "the hybrid needs a global max per stage");
    constexpr int H1 = MODE == 0 ? 1 : 2;
    constexpr int HALO = H1 * NST;
    constexpr int TILE = BS - 2 * HALO;
    constexpr int Q = K + 1;
    T* sTrR = reinterpret_cast<T*>(lds);                 // [NV][BS] right trace
    T* sF = sTrR + NV * BS;                             // [NV][BS] flux at left interface

    const int tid = threadIdx.x;
    const int64_t c = blk * TILE + tid - HALO;
    const int64_t n = a.n;
    bool valid = true;
    int64_t cc = c;
    if (c < 0 || c >= n) {
        if (a.periodic)
            cc = wrap(c, n);
        else
            valid = false;
    }

    double u0[NV], n0[NV];
    T uh[NV][KH], nh[NV][KH];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        u0[v] = n0[v] = 0.0;
#pragma unroll
        for (int l = 0; l < KH; ++l) uh[v][l] = nh[v][l] = (T)0;
    }
    if (valid) {
        if (NST == 1) {
            load_cell<K, NV, TB>(a.us, cc, u0, uh);
            if (a.stage > 0) load_cell<K, NV, TB>(a.un, cc, n0, nh);
            if (MODE == 2 && K > 0 && a.bl_us.eta && a.bl_un.eta) {
                // deferred blends owed by the inputs (u^n's is fetched at
                // stage 0 too, where both name the same slot)
                const auto bs = blend_fetch<K, TB>(a.bl_us, n, cc);
                const auto bn = blend_fetch<K, TB>(a.bl_un, n, cc);
                blend_pin(bs);
                blend_pin(bn);
                blend_apply<K, NV, TB>(bs, uh);
                if (a.stage > 0) blend_apply<K, NV, TB>(bn, nh);
            }
        } else {
            load_cell<K, NV, TB>(a.un, cc, n0, nh);
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                u0[v] = n0[v];
#pragma unroll
                for (int l = 0; l < KH; ++l) uh[v][l] = nh[v][l];
            }
        }
    }
    const bool own = valid && c >= 0 && c < n && tid >= HALO && tid < BS - HALO;
    double lam = 0.0;
    T eta_own = (T)0;
    // unrolled: the stage's coefficients and lane bounds become constants,
    // which keeps the fused kernels' register counts down
#pragma unroll
    for (int st = 0; st < NST; ++st) {
    const int stage = NST == 1 ? a.stage : st;
    // lanes whose stage input is valid, and those whose output will be
    const int in_lo = st * H1, in_hi = BS - 1 - st * H1;
    const bool last = st == NST - 1;
    // lanes whose output this stage produces: the final stage's own cells;
    // before it every valid lane in range (periodic halo lanes included)
    const bool own_s = last ? own : (valid && tid >= in_lo + H1 && tid <= in_hi - H1);
    if (st > 0) __syncthreads();  // the previous stage's LDS reads are complete
    // a fused step already flagged by the positivity limiter is discarded and
    // retried: its later stages may compute from an inadmissible state and
    // check nothing (every tile reading such a cell has flagged the step
    // itself, since it recomputes its halo, before this barrier)
    const bool chk = a.check && !(NST == 3 && st > 0 && a.reject &&
                                  __hip_atomic_load(a.reject, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));

    // Interface traces u(x^+_{j-1/2}) (left end) and u(x^-_{j+1/2}) (right end).
    T tl[NV], tr[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        T sl = (T)u0[v], sr = (T)u0[v];
#pragma unroll
        for (int l = 1; l <= K; ++l) {
            sr += uh[v][l - 1];
            sl += (l & 1) ? -uh[v][l - 1] : uh[v][l - 1];
        }
        tl[v] = sl;
        tr[v] = sr;
        sTrR[v * BS + tid] = sr;
    }

    // Positivity (Euler) of the stage input at the traces, in FP64.  The
    // FP64 path checks the pressures its interface fluxes compute instead.
    if (EQ == EULER && valid && chk && sizeof(T) != 8 && tid >= in_lo && tid <= in_hi) {
        double dl[NV], dr[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            double sl = u0[v], sr = u0[v];
#pragma unroll
            for (int l = 1; l <= K; ++l) {
                sr += (double)uh[v][l - 1];
                sl += (l & 1) ? -(double)uh[v][l - 1] : (double)uh[v][l - 1];
            }
            dl[v] = sl;
            dr[v] = sr;
        }
        double pl = Phys1D<EULER>::pressure(dl, a.phys), pr = Phys1D<EULER>::pressure(dr, a.phys);
        if (!(dl[0] > 0.0) || !(dr[0] > 0.0) || !(pl > 0.0) || !(pr > 0.0)) {
            bool fin = isfinite(dl[0]) && isfinite(dr[0]) && isfinite(pl) && isfinite(pr);
            // with the positivity limiter the traces sit at its margin up
            // to rounding; the limiter and the step rejection own positivity
            if (!fin || !a.pp) latch_error(a.ctrl, fin ? -5 : -4, cc);
        }
    }
    __syncthreads();

    // Flux at the left interface of this cell (once per interface).
    T fL[NV], fR[NV];
    if (valid && tid > in_lo && tid <= in_hi) {
        T left[NV];
        if (!a.periodic && c == 0) {
            ghost_state<NV, T>(a.bc_lo, a.dir_lo, tl, left);
        } else {
#pragma unroll
            for (int v = 0; v < NV; ++v) left[v] = sTrR[v * BS + tid - 1];
        }
        T pl, pr;
        llf1d<EQ, T, HLLX>(left, tl, fL, a.phys, &pl, &pr);
        if (EQ == EULER && chk && sizeof(T) == 8) trace_check(a, left, tl, pl, pr, cc);
#pragma unroll
        for (int v = 0; v < NV; ++v) sF[v * BS + tid] = fL[v];
    }
    __syncthreads();

    // Residual and Shu-Osher combination -> unfiltered output (v0, vh).
    const bool have_res = valid && tid >= in_lo + 1 && tid <= in_hi - 1;
    double v0[NV];
    T vh[NV][KH];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        v0[v] = 0.0;
#pragma unroll
        for (int l = 0; l < KH; ++l) vh[v][l] = (T)0;
    }
    if (have_res) {
        if (!a.periodic && c == n - 1) {
            T right[NV], pl, pr;
            ghost_state<NV, T>(a.bc_hi, a.dir_hi, tr, right);
            llf1d<EQ, T, HLLX>(tr, right, fR, a.phys, &pl, &pr);
            if (EQ == EULER && chk && sizeof(T) == 8) trace_check(a, tr, right, pl, pr, cc);
        } else {
#pragma unroll
            for (int v = 0; v < NV; ++v) fR[v] = sF[v * BS + tid + 1];
        }
        // Boundary fluxes for the conservation ledger (one writer each).
        if (a.bflux && !a.periodic && tid >= HALO && tid < BS - HALO) {
            double* bf = a.bflux + (NST == 1 ? 0 : 8 * st);
            // atomic stores: the step control may run in another workgroup
            // of this launch and read them at the point of coherence
            if (c == 0)
#pragma unroll
                for (int v = 0; v < NV; ++v) store_coherent(&bf[v], (double)fL[v]);
            if (c == n - 1)
#pragma unroll
                for (int v = 0; v < NV; ++v) store_coherent(&bf[4 + v], (double)fR[v]);
        }
        // Volume term: int f(u_h) P_l'(xi) dxi by the (K+1)-point Gauss rule.
        T vol[NV][KH];
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int l = 0; l < KH; ++l) vol[v][l] = (T)0;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            T uq[NV], fq[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                T s = (T)u0[v];
#pragma unroll
                for (int l = 1; l <= K; ++l) s += uh[v][l - 1] * (T)leg_at(Q, q, l);
                uq[v] = s;
            }
            const T pq = P::flux_pressure(uq, fq, a.phys);
            if (EQ == EULER && chk && valid) {
                if (!(uq[0] > (T)0) || !(pq > (T)0)) {
                    bool fin = isfinite((double)uq[0]) && isfinite((double)pq);
                    latch_error(a.ctrl, fin ? -5 : -4, cc);
                }
            }
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                T wf = (T)gl_weight(Q, q) * fq[v];
#pragma unroll
                for (int l = 1; l <= K; ++l) vol[v][l - 1] += wf * (T)dleg_at(Q, q, l);
            }
        }
        const T ih = (T)a.inv_h;
        const T tdt = (T)dt;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            // mode 0: P_0' = 0, flux difference of the shared FP32/FP64
            // interface fluxes accumulated in FP64 (conservative)
            double L0 = -((double)fR[v] - (double)fL[v]) * a.inv_h;
            v0[v] = combine(stage, n0[v], u0[v] + dt * L0);
#pragma unroll
            for (int l = 1; l <= K; ++l) {
                T fl = (l & 1) ? -fL[v] : fL[v];
                T L = (T)(2 * l + 1) * ih * (vol[v][l - 1] - fR[v] + fl);
                vh[v][l - 1] = combine_t<T>(stage, nh[v][l - 1], uh[v][l - 1] + tdt * L);
            }
        }
    }

    if constexpr (MODE == 0) {
        if (last) {
            if (own) {
                lam = finish_cell<EQ, K, TB, NV>(a, c, v0, vh, true);
                store_cell<K, NV, TB>(a.out, c, v0, vh);
            }
        } else {
            // an intermediate stage of a fused step: the limiter as the
            // single-stage kernel applies it to its output
            if (own_s) finish_cell<EQ, K, TB, NV>(a, c, v0, vh, true);
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                u0[v] = v0[v];
#pragma unroll
                for (int l = 0; l < KH; ++l) uh[v][l] = vh[v][l];
            }
        }
    } else {
        // ---- jump filter on the unfiltered output (needs neighbours) ----
        __syncthreads();  // phase-1 LDS reads are complete
        double* s0 = reinterpret_cast<double*>(lds);       // [NV][BS] mode 0
        T* sHR = reinterpret_cast<T*>(s0 + NV * BS);      // [K1][NV][BS] right high-mode part
        T* sJ = sHR;                                      // then: jumps at the left interface
        T hR[K1][NV], hL[K1][NV];
#pragma unroll
        for (int m = 0; m <= K; ++m)
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                T r = (T)0, l_ = (T)0;
#pragma unroll
                for (int l = (m > 1 ? m : 1); l <= K; ++l) {
                    r += vh[v][l - 1] * (T)dtrace_r(l, m);
                    l_ += vh[v][l - 1] * (T)dtrace_l(l, m);
                }
                hR[m][v] = r;
                hL[m][v] = l_;
                sHR[(m * NV + v) * BS + tid] = r;
            }
#pragma unroll
        for (int v = 0; v < NV; ++v) s0[v * BS + tid] = v0[v];
        __syncthreads();

        // |[d^m u]| at the left interface of lanes 1..BS-2 (the own cells and
        // the first halo lane on the right): each interface jump is formed
        // once, by the cell to its right, and handed to its left neighbour
        // through LDS
        const bool lbound = !a.periodic && c == 0, rbound = !a.periodic && c == n - 1;
        const bool jlane = tid >= in_lo + 2 && tid <= in_hi - 1;
        T jl[K1][NV];
#pragma unroll
        for (int m = 0; m <= K; ++m)
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                jl[m][v] = (T)0;
                if (!jlane) continue;
                if (lbound) {
                    T inner = (m == 0 ? (T)v0[v] : (T)0) + hL[m][v];
                    jl[m][v] = ghost_jump<T>(a.bc_lo, m, v, a.dir_lo[v], inner);
                } else {
                    T d = hL[m][v] - sHR[(m * NV + v) * BS + tid - 1];
                    if (m == 0) d += (T)(v0[v] - s0[v * BS + tid - 1]);
                    jl[m][v] = fabs(d);
                }
            }
        __syncthreads();  // the right traces are consumed
        if (jlane) {
#pragma unroll
            for (int m = 0; m <= K; ++m)
#pragma unroll
                for (int v = 0; v < NV; ++v) sJ[(m * NV + v) * BS + tid] = jl[m][v];
        }
        __syncthreads();

        if (own_s) {
            // S[l][v] = sum_{m<=l} m(m+1) 2^m (|[d^m]|_left + |[d^m]|_right)
            T J[K1][NV];
#pragma unroll
            for (int m = 0; m <= K; ++m)
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    T jr;
                    if (rbound) {
                        T inner = (m == 0 ? (T)v0[v] : (T)0) + hR[m][v];
                        jr = ghost_jump<T>(a.bc_hi, m, v, a.dir_hi[v], inner);
                    } else {
                        jr = sJ[(m * NV + v) * BS + tid + 1];
                    }
                    J[m][v] = jl[m][v] + jr;
                }
            // beta_j = |f'(u-bar_j)|, H-bar_j from the cell average; the
            // exponent sigma_j^l dt = beta dt / (h H) * max_s S^l_s (the
            // l(l+1) of c_f^l and of (2/h)^2 l(l+1) cancel).
            T ub[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) ub[v] = (T)v0[v];
            const T beta = P::speed(ub, a.phys);
            const T H = P::enthalpy(ub, a.phys);
            const T coef = beta * (T)dt * (T)a.inv_h * trcp<T>(H);
            T E[K1];
            E[0] = (T)0;
            T S[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) S[v] = J[0][v];
#pragma unroll
            for (int l = 1; l <= K; ++l) {
                T mx = (T)0;
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    S[v] += (T)jump_weight(l) * J[l][v];
                    mx = (v == 0 || S[v] > mx) ? S[v] : mx;
                }
                E[l] = coef * mx;
            }
            T eta = (T)0;
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                T e = J[0][v] * (T)(0.5 * a.inv_h);
                eta = (v == 0 || e > eta) ? e : eta;
            }
            eta_own = eta;

            if constexpr (MODE == 1) {
#pragma unroll
                for (int l = 1; l <= K; ++l) {
                    T f = texp<T>(-E[l]);
#pragma unroll
                    for (int v = 0; v < NV; ++v) vh[v][l - 1] *= f;
                }
                if (last) {
                    lam = finish_cell<EQ, K, TB, NV>(a, c, v0, vh, true);
                    store_cell<K, NV, TB>(a.out, c, v0, vh);
                } else {
                    finish_cell<EQ, K, TB, NV>(a, c, v0, vh, true);
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        u0[v] = v0[v];
#pragma unroll
                        for (int l = 0; l < KH; ++l) uh[v][l] = vh[v][l];
                    }
                }
            } else {
                // troubled cells are limited after the blend (pass B)
                lam = finish_cell<EQ, K, TB, NV>(a, c, v0, vh, !(eta > (T)1));
                store_cell<K, NV, TB>(a.out, c, v0, vh);
                if (a.dv_eta) {
                    // pass B deferred to the next reader of this output
                    a.dv_eta[c] = (TB)eta;
                    if (eta > (T)1) {
                        atomicAdd(a.tcount, 1u);
#pragma unroll
                        for (int l = 1; l <= K; ++l) a.dv_E[(int64_t)(l - 1) * n + c] = (TB)E[l];
                    }
                } else if (eta > (T)1) {
                    unsigned int slot = atomicAdd(a.tcount, 1u);
                    if ((long long)slot < a.tcap) {
                        a.tcell[slot] = c;
                        double* rec = a.tdata + (size_t)slot * K1;
                        rec[0] = (double)eta;
#pragma unroll
                        for (int l = 1; l <= K; ++l) rec[l] = (double)E[l];
                    }
                }
            }
            if (a.E_out && last) {
#pragma unroll
                for (int l = 0; l <= K; ++l) a.E_out[c * K1 + l] = (double)E[l];
            }
        }
    }
    }  // stages
    *eta_out = (double)eta_own;
    // CFL quantity of the output (FP64): its cell average, and with the
    // positivity limiter also the test points
    *lam_out = lam;
}

// Hybrid pass B over entries i0, i0+stride, ... of the troubled list:
// u^l <- [omega + (1 - omega) exp(-E^l)] u^l, omega = (M - eta) / (M - 1),
// M = max eta; then, with the positivity limiter on, the limiter on the
// blended cell.
template <int K, int NV, typename TB>
__device__ __forceinline__ void blend_entries(StateView<TB> out, unsigned int cnt, const long long* tcell,
                                              const double* tdata, unsigned long long eta_bits,
                                              long long cap, const PPArgs& pp, unsigned int i0,
                                              unsigned int stride)
{
    if ((long long)cnt > cap) cnt = (unsigned int)cap;
    const double M = __longlong_as_double((long long)eta_bits);
    for (unsigned int i = i0; i < cnt; i += stride) {
        const long long c = tcell[i];
        const double* rec = tdata + (size_t)i * (K + 1);
        const double eta = rec[0];
        const double w = (M - eta) / (M - 1.0);
#pragma unroll
        for (int l = 1; l <= K; ++l) {
            const TB f = (TB)(w + (1.0 - w) * exp(-rec[l]));
#pragma unroll
            for (int v = 0; v < NV; ++v) out.hi[v * out.sv + (l - 1) * out.sl + c] *= f;
        }
        if constexpr (NV == 3) {
            if (pp.on) {
                double v0[3];
                TB vh[3][K > 0 ? K : 1];
                load_cell<K, 3, TB>(out, c, v0, vh);
                pp_limit<K, TB>(v0, vh, pp.phys.gamma);
                if (!pp_admissible(v0, pp.phys.gamma) && pp.reject) atomicOr(pp.reject, 1);
                store_cell<K, 3, TB>(out, c, v0, vh);
            }
        }
    }
}

// Tile of this workgroup.  Workgroups are dealt to the 8 XCDs round-robin;
// each XCD takes one contiguous range of tiles, so neighbouring tiles, which
// read each other's edge cells, mostly run on the same XCD and its L2.
__device__ __forceinline__ int64_t xcd_block()
{
    const int64_t p = blockIdx.x, q = gridDim.x >> 3, r = gridDim.x & 7;
    const int64_t x = p & 7, k = p >> 3;
    return x * q + (x < r ? x : r) + k;
}

// FOLD: the last workgroup to finish runs the next step's control (built for
// the small-grid hybrid stage only, BS = 128: it raises the kernel's register
// count).
template <int EQ, int K, typename TB, int MODE, int BS, bool HLLX, int NST, bool FOLD = false>
__global__ __launch_bounds__(BS) void stage1d_kernel(Args1D<TB> a)
{
    // a finished run, or a step already rejected by the positivity limiter;
    // both flags are read in one trip to memory (the host code sets a.ctrl
    // for every launch)
    const Ctrl* c = a.ctrl;
    const int flags = c->done | c->reject;
    if (a.dt_from_ctrl && flags) return;
    const double dt = a.dt_from_ctrl ? c->dt : a.dt_host;
    if (a.zero_bits && blockIdx.x == 0 && threadIdx.x == 0) *a.zero_bits = 0;
    __shared__ __align__(16) unsigned char lds[Stage1DLds<EQ, K, TB, MODE, BS>::bytes];
    double lam, eta;
    stage1d_tile<EQ, K, TB, MODE, BS, HLLX, NST>(a, xcd_block(), dt, lds, &lam, &eta);
    if (MODE == 2) {
        // max eta over the domain (wave reduction, one atomic per wave)
        const double e = wave_max(eta);
        if ((threadIdx.x & 63) == 0) atomic_max_nonneg(a.eta_acc, e);
    }
    if (a.alpha_acc) {
        // CFL reduction of the output's cell averages (next step)
        const double l = wave_max(lam);
        if ((threadIdx.x & 63) == 0) atomic_max_nonneg(a.alpha_acc, l);
    }
    if constexpr (FOLD) {
        // the next step's control, run by the workgroup that finishes last:
        // each workgroup waits for its own memory operations (its atomics
        // into the control block are then performed) before counting itself in
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (threadIdx.x == 0 &&
            __hip_atomic_fetch_add(&a.ctrl->arrive.v, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
                (unsigned long long)gridDim.x - 1)
            step_ctrl_in_kernel(a.ctrl);
    }
}

// Hybrid pass B as a kernel of its own (per-call path and the dg_run graph
// with the positivity limiter on).
template <int K, int NV, typename TB>
__global__ __launch_bounds__(256) void blend1d_kernel(StateView<TB> out, const unsigned int* count,
                                                      const long long* tcell, const double* tdata,
                                                      const unsigned long long* eta_bits,
                                                      const Ctrl* ctrl, int from_ctrl, long long cap,
                                                      PPArgs pp)
{
    // the control flags, the list length and the maximum are fetched
    // together (one memory round trip) before anything depends on them
    const int stop = from_ctrl ? (ctrl->done | ctrl->reject) : 0;
    const unsigned int cnt = *count;
    const unsigned long long eb = *eta_bits;
    if (stop) return;
    blend_entries<K, NV, TB>(out, cnt, tcell, tdata, eb, cap, pp, blockIdx.x * blockDim.x + threadIdx.x,
                             gridDim.x * blockDim.x);
}

// The blend a state still owes (deferred hybrid pass B), applied in place.
template <int K, int NV, typename TB>
__global__ __launch_bounds__(256) void deferred_blend_kernel(StateView<TB> u, int64_t n,
                                                             typename Args1D<TB>::Deferred bl)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    double u0[NV];
    TB uh[NV][K > 0 ? K : 1];
    load_cell<K, NV, TB>(u, c, u0, uh);
    blend_apply<K, NV, TB>(blend_fetch<K, TB>(bl, n, c), uh);
    store_cell<K, NV, TB>(u, c, u0, uh);
}

// Unfused filter / hybrid (per-call API): reads the unfiltered stage output
// w (halo 1) and either writes the filtered result (MODE 1) or the
// exponents and eta per cell (MODE 2, followed by blend_all1d_kernel).
template <int EQ, int K, typename TB, int MODE>
__global__ __launch_bounds__(256) void filter1d_kernel(Args1D<TB> a)
{
    using P = Phys1D<EQ>;
    using T = TB;
    constexpr int NV = P::NV;
    constexpr int K1 = K + 1;
    constexpr int KH = K > 0 ? K : 1;
    constexpr int TILE = 254;
    const double dt = a.dt_host;

    __shared__ __align__(16) double s0[NV * 256];
    __shared__ __align__(16) T sHR[K1 * NV * 256];
    __shared__ __align__(16) T sHL[K1 * NV * 256];

    const int tid = threadIdx.x;
    const int64_t c = (int64_t)blockIdx.x * TILE + tid - 1;
    const int64_t n = a.n;
    bool valid = true;
    int64_t cc = c;
    if (c < 0 || c >= n) {
        if (a.periodic)
            cc = wrap(c, n);
        else
            valid = false;
    }
    double v0[NV];
    T vh[NV][KH];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        v0[v] = 0.0;
#pragma unroll
        for (int l = 0; l < KH; ++l) vh[v][l] = (T)0;
    }
    if (valid) load_cell<K, NV, TB>(a.us, cc, v0, vh);

    T hR[K1][NV], hL[K1][NV];
#pragma unroll
    for (int m = 0; m <= K; ++m)
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            T r = (T)0, l_ = (T)0;
#pragma unroll
            for (int l = (m > 1 ? m : 1); l <= K; ++l) {
                r += vh[v][l - 1] * (T)dtrace_r(l, m);
                l_ += vh[v][l - 1] * (T)dtrace_l(l, m);
            }
            hR[m][v] = r;
            hL[m][v] = l_;
            sHR[(m * NV + v) * 256 + tid] = r;
            sHL[(m * NV + v) * 256 + tid] = l_;
        }
#pragma unroll
    for (int v = 0; v < NV; ++v) s0[v * 256 + tid] = v0[v];
    __syncthreads();

    const bool own = valid && c >= 0 && c < n && tid >= 1 && tid <= 254;
    if (!own) return;
    T J[K1][NV];
    const bool lbound = !a.periodic && c == 0, rbound = !a.periodic && c == n - 1;
#pragma unroll
    for (int m = 0; m <= K; ++m)
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            T jl, jr;
            if (lbound) {
                T inner = (m == 0 ? (T)v0[v] : (T)0) + hL[m][v];
                jl = ghost_jump<T>(a.bc_lo, m, v, a.dir_lo[v], inner);
            } else {
                T d = hL[m][v] - sHR[(m * NV + v) * 256 + tid - 1];
                if (m == 0) d += (T)(v0[v] - s0[v * 256 + tid - 1]);
                jl = fabs(d);
            }
            if (rbound) {
                T inner = (m == 0 ? (T)v0[v] : (T)0) + hR[m][v];
                jr = ghost_jump<T>(a.bc_hi, m, v, a.dir_hi[v], inner);
            } else {
                T d = sHL[(m * NV + v) * 256 + tid + 1] - hR[m][v];
                if (m == 0) d += (T)(s0[v * 256 + tid + 1] - v0[v]);
                jr = fabs(d);
            }
            J[m][v] = jl + jr;
        }
    T ub[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) ub[v] = (T)v0[v];
    const T beta = P::speed(ub, a.phys);
    const T H = P::enthalpy(ub, a.phys);
    const T coef = beta * (T)dt * (T)a.inv_h * trcp<T>(H);
    T E[K1];
    E[0] = (T)0;
    T S[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) S[v] = J[0][v];
#pragma unroll
    for (int l = 1; l <= K; ++l) {
        T mx = (T)0;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            S[v] += (T)jump_weight(l) * J[l][v];
            mx = (v == 0 || S[v] > mx) ? S[v] : mx;
        }
        E[l] = coef * mx;
    }
    T eta = (T)0;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        T e = J[0][v] * (T)(0.5 * a.inv_h);
        eta = (v == 0 || e > eta) ? e : eta;
    }
    if (a.E_out) {
#pragma unroll
        for (int l = 0; l <= K; ++l) a.E_out[c * K1 + l] = (double)E[l];
    }
    if constexpr (MODE == 1) {
#pragma unroll
        for (int l = 1; l <= K; ++l) {
            T f = texp<T>(-E[l]);
#pragma unroll
            for (int v = 0; v < NV; ++v) vh[v][l - 1] *= f;
        }
        finish_cell<EQ, K, TB, NV>(a, c, v0, vh, true);
        store_cell<K, NV, TB>(a.out, c, v0, vh);
    } else {
        a.eta_out[c] = (double)eta;
        atomic_max_nonneg(a.eta_acc, (double)eta);
    }
}

// Hybrid blend over all cells (per-call API): out = w for calm cells, the
// blended polynomial for troubled ones.
template <int K, int NV, typename TB>
__global__ __launch_bounds__(256) void blend_all1d_kernel(StateView<TB> w, StateView<TB> out, int64_t n,
                                                          const double* E, const double* eta,
                                                          const unsigned long long* eta_bits,
                                                          unsigned int* tcount, PPArgs pp)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    constexpr int KH = K > 0 ? K : 1;
    double v0[NV];
    TB vh[NV][KH];
    load_cell<K, NV, TB>(w, c, v0, vh);
    // eta == nullptr: no hybrid blend (the limiter alone, after a plain stage)
    const double M = eta ? __longlong_as_double((long long)*eta_bits) : 0.0;
    const double e = eta ? eta[c] : 0.0;
    if (e > 1.0) {
        atomicAdd(tcount, 1u);
        const double om = (M - e) / (M - 1.0);
#pragma unroll
        for (int l = 1; l <= K; ++l) {
            const TB f = (TB)(om + (1.0 - om) * exp(-E[c * (K + 1) + l]));
#pragma unroll
            for (int v = 0; v < NV; ++v) vh[v][l - 1] *= f;
        }
    }
    if constexpr (NV == 3) {
        if (pp.on) {
            pp_limit<K, TB>(v0, vh, pp.phys.gamma);
            if (!pp_admissible(v0, pp.phys.gamma) && pp.reject) atomicOr(pp.reject, 1);
        }
    }
    store_cell<K, NV, TB>(out, c, v0, vh);
}

// CFL reduction over the cell averages of u (FP64).
template <int EQ, typename TB>
__global__ __launch_bounds__(256) void maxwave1d_kernel(StateView<TB> u, int64_t n, PhysParams phys,
                                                        unsigned long long* acc, Ctrl* err)
{
    constexpr int NV = Phys1D<EQ>::NV;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double lam = 0.0;
    if (c < n) {
        double ub[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) ub[v] = u.m0[v * u.s0 + c];
        lam = Phys1D<EQ>::speed(ub, phys);
        if (EQ == EULER) {
            const double p = Phys1D<EULER>::pressure(ub, phys);
            if (!(ub[0] > 0.0) || !(p > 0.0))
                latch_error(err, (isfinite(ub[0]) && isfinite(p)) ? -5 : -4, c);
        }
        if (!isfinite(lam)) latch_error(err, -4, c);
    }
    lam = wave_max(lam);
    if ((threadIdx.x & 63) == 0) atomic_max_nonneg(acc, lam);
}

// ------------------------------------------------------------ launchers --
// nst = 1: one RK stage (a.stage); nst = 3: the whole step (MODE 0 or 1).
// BS = 128 is built for the hybrid stage only.
template <int EQ, int K, typename TB, int BS, bool HLLX>
static hipError_t launch_stage_fx(const Args1D<TB>& a, int mode, int nst, hipStream_t st)
{
    const int tile = BS - 2 * nst * (mode == 0 ? 1 : 2);
    dim3 grid((unsigned)((a.n + tile - 1) / tile)), block(BS);
    if constexpr (BS == 128) {
        if (mode != 2 || nst != 1) return hipErrorInvalidValue;
        if (a.fold_ctrl)
            hipLaunchKernelGGL((stage1d_kernel<EQ, K, TB, 2, BS, HLLX, 1, true>), grid, block, 0, st, a);
        else
            hipLaunchKernelGGL((stage1d_kernel<EQ, K, TB, 2, BS, HLLX, 1>), grid, block, 0, st, a);
        return hipGetLastError();
    }
    if (nst == 3) {
        if (mode == 0)
            hipLaunchKernelGGL((stage1d_kernel<EQ, K, TB, 0, BS, HLLX, 3>), grid, block, 0, st, a);
        else if (mode == 1)
            hipLaunchKernelGGL((stage1d_kernel<EQ, K, TB, 1, BS, HLLX, 3>), grid, block, 0, st, a);
        else
            return hipErrorInvalidValue;
    } else if (mode == 0)
        hipLaunchKernelGGL((stage1d_kernel<EQ, K, TB, 0, BS, HLLX, 1>), grid, block, 0, st, a);
    else if (mode == 1)
        hipLaunchKernelGGL((stage1d_kernel<EQ, K, TB, 1, BS, HLLX, 1>), grid, block, 0, st, a);
    else if (!a.fold_ctrl)
        hipLaunchKernelGGL((stage1d_kernel<EQ, K, TB, 2, BS, HLLX, 1>), grid, block, 0, st, a);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// The HLL family of fluxes (Euler) has kernels of its own.
template <int EQ, int K, typename TB, int BS>
static hipError_t launch_stage_bs(const Args1D<TB>& a, int mode, int nst, hipStream_t st)
{
    if constexpr (EQ == EULER)
        if (a.phys.flux != FLUX_LLF) return launch_stage_fx<EQ, K, TB, BS, true>(a, mode, nst, st);
    return launch_stage_fx<EQ, K, TB, BS, false>(a, mode, nst, st);
}

// Small grids (under about a thousand 256-cell tiles) use small tiles: a
// single tile's dependent chain then bounds the stage, and smaller tiles
// spread it over more compute units.  The hybrid stage takes two-wavefront
// tiles (measured faster than one- or four-wavefront ones there), the rest
// one-wavefront tiles.
template <int EQ, int K, typename TB>
static hipError_t launch_stage(const Args1D<TB>& a, int mode, int nst, hipStream_t st)
{
    if (a.n < kSmallTileCells) {
        if (mode == 2 && nst == 1) return launch_stage_bs<EQ, K, TB, 128>(a, mode, nst, st);
        return launch_stage_bs<EQ, K, TB, 64>(a, mode, nst, st);
    }
    return launch_stage_bs<EQ, K, TB, 256>(a, mode, nst, st);
}

template <int EQ, int K, typename TB>
static hipError_t launch_filter(const Args1D<TB>& a, int mode, hipStream_t st)
{
    dim3 grid((unsigned)((a.n + 253) / 254)), block(256);
    if (mode == 1)
        hipLaunchKernelGGL((filter1d_kernel<EQ, K, TB, 1>), grid, block, 0, st, a);
    else
        hipLaunchKernelGGL((filter1d_kernel<EQ, K, TB, 2>), grid, block, 0, st, a);
    return hipGetLastError();
}

template <typename TB>
hipError_t launch_stage1d(int eq, int k, const Args1D<TB>& a, int mode, hipStream_t st, int nst)
{
#define DG_CASE(E_, K_) \
    if (eq == E_ && k == K_) return launch_stage<E_, K_, TB>(a, mode, nst, st);
    DG_CASE(ADV, 0) DG_CASE(ADV, 1) DG_CASE(ADV, 2) DG_CASE(ADV, 3)
    DG_CASE(BURGERS, 0) DG_CASE(BURGERS, 1) DG_CASE(BURGERS, 2) DG_CASE(BURGERS, 3)
    DG_CASE(EULER, 0) DG_CASE(EULER, 1) DG_CASE(EULER, 2) DG_CASE(EULER, 3)
#undef DG_CASE
    return hipErrorInvalidValue;
}

template <typename TB>
hipError_t launch_filter1d(int eq, int k, const Args1D<TB>& a, int mode, hipStream_t st)
{
#define DG_CASE(E_, K_) \
    if (eq == E_ && k == K_) return launch_filter<E_, K_, TB>(a, mode, st);
    DG_CASE(ADV, 0) DG_CASE(ADV, 1) DG_CASE(ADV, 2) DG_CASE(ADV, 3)
    DG_CASE(BURGERS, 0) DG_CASE(BURGERS, 1) DG_CASE(BURGERS, 2) DG_CASE(BURGERS, 3)
    DG_CASE(EULER, 0) DG_CASE(EULER, 1) DG_CASE(EULER, 2) DG_CASE(EULER, 3)
#undef DG_CASE
    return hipErrorInvalidValue;
}

template <typename TB>
hipError_t launch_blend1d(int nv, int k, StateView<TB> out, const unsigned int* count,
                          const long long* tcell, const double* tdata,
                          const unsigned long long* eta_bits, const Ctrl* ctrl, int from_ctrl,
                          int64_t max_entries, PPArgs pp, hipStream_t st)
{
    unsigned g = (unsigned)((max_entries + 255) / 256);
    if (g > 1024) g = 1024;
    if (g < 1) g = 1;
#define DG_CASE(NV_, K_)                                                                            \
    if (nv == NV_ && k == K_) {                                                                     \
        hipLaunchKernelGGL((blend1d_kernel<K_, NV_, TB>), dim3(g), dim3(256), 0, st, out, count,      \
                           tcell, tdata, eta_bits, ctrl, from_ctrl, (long long)max_entries, pp);   \
        return hipGetLastError();                                                                   \
    }
    DG_CASE(1, 0) DG_CASE(1, 1) DG_CASE(1, 2) DG_CASE(1, 3)
    DG_CASE(3, 0) DG_CASE(3, 1) DG_CASE(3, 2) DG_CASE(3, 3)
#undef DG_CASE
    return hipErrorInvalidValue;
}

template <typename TB>
hipError_t launch_deferred_blend1d(int nv, int k, StateView<TB> u, int64_t n,
                                   typename Args1D<TB>::Deferred bl, hipStream_t st)
{
    dim3 grid((unsigned)((n + 255) / 256)), block(256);
#define DG_CASE(NV_, K_)                                                                          \
    if (nv == NV_ && k == K_) {                                                                   \
        hipLaunchKernelGGL((deferred_blend_kernel<K_, NV_, TB>), grid, block, 0, st, u, n, bl);   \
        return hipGetLastError();                                                                 \
    }
    DG_CASE(1, 0) DG_CASE(1, 1) DG_CASE(1, 2) DG_CASE(1, 3)
    DG_CASE(3, 0) DG_CASE(3, 1) DG_CASE(3, 2) DG_CASE(3, 3)
#undef DG_CASE
    return hipErrorInvalidValue;
}

template <typename TB>
hipError_t launch_blend_all1d(int nv, int k, StateView<TB> w, StateView<TB> out, int64_t n,
                              const double* E, const double* eta,
                              const unsigned long long* eta_bits, unsigned int* tcount,
                              PPArgs pp, hipStream_t st)
{
    dim3 grid((unsigned)((n + 255) / 256)), block(256);
#define DG_CASE(NV_, K_)                                                                           \
    if (nv == NV_ && k == K_) {                                                                    \
        hipLaunchKernelGGL((blend_all1d_kernel<K_, NV_, TB>), grid, block, 0, st, w, out, n, E, eta, \
                           eta_bits, tcount, pp);                                                  \
        return hipGetLastError();                                                                  \
    }
    DG_CASE(1, 0) DG_CASE(1, 1) DG_CASE(1, 2) DG_CASE(1, 3)
    DG_CASE(3, 0) DG_CASE(3, 1) DG_CASE(3, 2) DG_CASE(3, 3)
#undef DG_CASE
    return hipErrorInvalidValue;
}

template <typename TB>
hipError_t launch_maxwave1d(int eq, StateView<TB> u, int64_t n, PhysParams phys,
                            unsigned long long* acc, Ctrl* err, hipStream_t st)
{
    dim3 grid((unsigned)((n + 255) / 256)), block(256);
    if (eq == ADV)
        hipLaunchKernelGGL((maxwave1d_kernel<ADV, TB>), grid, block, 0, st, u, n, phys, acc, err);
    else if (eq == BURGERS)
        hipLaunchKernelGGL((maxwave1d_kernel<BURGERS, TB>), grid, block, 0, st, u, n, phys, acc, err);
    else
        hipLaunchKernelGGL((maxwave1d_kernel<EULER, TB>), grid, block, 0, st, u, n, phys, acc, err);
    return hipGetLastError();
}

#define DG_INST(TB)                                                                                 \
    template hipError_t launch_stage1d<TB>(int, int, const Args1D<TB>&, int, hipStream_t, int);     \
    template hipError_t launch_filter1d<TB>(int, int, const Args1D<TB>&, int, hipStream_t);         \
    template hipError_t launch_blend1d<TB>(int, int, StateView<TB>, const unsigned int*,            \
                                           const long long*, const double*,                        \
                                           const unsigned long long*, const Ctrl*, int, int64_t,   \
                                           PPArgs, hipStream_t);                                   \
    template hipError_t launch_deferred_blend1d<TB>(int, int, StateView<TB>, int64_t,              \
                                                    typename Args1D<TB>::Deferred, hipStream_t);   \
    template hipError_t launch_blend_all1d<TB>(int, int, StateView<TB>, StateView<TB>, int64_t,     \
                                               const double*, const double*,                       \
                                               const unsigned long long*, unsigned int*, PPArgs,   \
                                               hipStream_t);                                       \
    template hipError_t launch_maxwave1d<TB>(int, StateView<TB>, int64_t, PhysParams,               \
                                             unsigned long long*, Ctrl*, hipStream_t);
DG_INST(double)
DG_INST(float)
#undef DG_INST

}  // namespace dg
#include "dg_batch_kernel.h"
