// dg2d.hip — 2D Q^k RKDG stage, jump filter, hybrid limiter and CFL
// kernels for gfx950 (arXiv:2407.19169, Sec. 2.3 two-dimensional scheme and
// filter, Sec. 2.4 systems, Sec. 3 Algorithm 1).
//
// Mapping: one lane per (cell, variable), the variables of a cell in
// adjacent lanes; 16 x (256 / (16 NV)) cells per 256-thread workgroup (16x4
// for Euler); x-fastest SoA mode planes.  Tiles are staged in LDS with the
// neighbour cells they need, found by global cell coordinate (wrapped when
// periodic, flagged when outside the domain), so ragged tiles need no
// special case.
//   stage2d:  each lane publishes its variable's edge traces; every
//             (edge, Gauss point) flux is evaluated once per tile; the volume
//             fluxes are shared among the lanes of a cell, one Gauss point of
//             the current row per lane.
//   filter2d: the jumps of every mixed derivative at the two corners of each
//             edge are sum-factorised contractions of the two cells' modes
//             with the derivative values P_p^(a)(+-1), per variable; the
//             maximum over the variables is taken inside the cell's lanes.
#include <type_traits>

#include "dg_kernels.h"

namespace dg {

namespace {

template <int EQ>
struct Phys2D;

template <>
struct Phys2D<ADV> {
    static constexpr int NV = 1;
    template <typename T>
    __device__ static void flux(const T* u, int dir, T* f, const PhysParams& p)
    {
        f[0] = (T)p.a[dir] * u[0];
    }
    template <typename T>
    __device__ static T speed(const T* u, int dir, const PhysParams& p) { return fabs((T)p.a[dir]); }
    // CFL quantity speed_x / hx + speed_y / hy
    template <typename T>
    __device__ static T cfl(const T* u, T ihx, T ihy, const PhysParams& p)
    {
        return fabs((T)p.a[0]) * ihx + fabs((T)p.a[1]) * ihy;
    }
    template <typename T>
    __device__ static T enthalpy(const T* u, const PhysParams& p) { return (T)1; }
};

template <>
struct Phys2D<EULER> {
    static constexpr int NV = 4;
    template <typename T>
    __device__ static T pressure(const T* u, const PhysParams& p)
    {
        return ((T)p.gamma - (T)1) * (u[3] - (T)0.5 * (u[1] * u[1] + u[2] * u[2]) / u[0]);
    }
    template <typename T>
    __device__ static void flux(const T* u, int dir, T* f, const PhysParams& p)
    {
        const T ir = trcp<T>(u[0]);
        const T vx = u[1] * ir, vy = u[2] * ir;
        const T pr = ((T)p.gamma - (T)1) * (u[3] - (T)0.5 * (u[1] * vx + u[2] * vy));
        const T vn = dir == 0 ? vx : vy;
        f[0] = u[0] * vn;
        f[1] = u[1] * vn + (dir == 0 ? pr : (T)0);
        f[2] = u[2] * vn + (dir == 1 ? pr : (T)0);
        f[3] = vn * (u[3] + pr);
    }
    // (speed, enthalpy and the CFL quantity each from one reciprocal of the density)
    template <typename T>
    __device__ static T speed(const T* u, int dir, const PhysParams& p)
    {
        const T ir = trcp<T>(u[0]);
        const T vx = u[1] * ir, vy = u[2] * ir;
        const T pr = ((T)p.gamma - (T)1) * (u[3] - (T)0.5 * (u[1] * vx + u[2] * vy));
        return fabs(dir == 0 ? vx : vy) + tsqrt<T>((T)p.gamma * pr * ir);
    }
    template <typename T>
    __device__ static T cfl(const T* u, T ihx, T ihy, const PhysParams& p)
    {
        const T ir = trcp<T>(u[0]);
        const T vx = u[1] * ir, vy = u[2] * ir;
        const T pr = ((T)p.gamma - (T)1) * (u[3] - (T)0.5 * (u[1] * vx + u[2] * vy));
        const T c = tsqrt<T>((T)p.gamma * pr * ir);
        return (fabs(vx) + c) * ihx + (fabs(vy) + c) * ihy;
    }
    // flux() and speed() of one state from one reciprocal of the density
    template <typename T>
    __device__ static T flux_speed(const T* u, int dir, T* f, const PhysParams& p)
    {
        const T ir = trcp<T>(u[0]);
        const T vx = u[1] * ir, vy = u[2] * ir;
        const T pr = ((T)p.gamma - (T)1) * (u[3] - (T)0.5 * (u[1] * vx + u[2] * vy));
        const T vn = dir == 0 ? vx : vy;
        f[0] = u[0] * vn;
        f[1] = u[1] * vn + (dir == 0 ? pr : (T)0);
        f[2] = u[2] * vn + (dir == 1 ? pr : (T)0);
        f[3] = vn * (u[3] + pr);
        return fabs(vn) + tsqrt<T>((T)p.gamma * pr * ir);
    }
    template <typename T>
    __device__ static T enthalpy(const T* u, const PhysParams& p)
    {
        const T ir = trcp<T>(u[0]);
        const T pr = ((T)p.gamma - (T)1) * (u[3] - (T)0.5 * (u[1] * (u[1] * ir) + u[2] * (u[2] * ir)));
        return (u[3] + pr) * ir;
    }
};

// Interface flux across a face of normal +dir: local Lax-Friedrichs (the
// default) or, in Euler kernels compiled with HLLX, HLL / HLLC (p.flux).
template <int EQ, typename T, bool HLLX = false>
__device__ __forceinline__ void llf2d(const T* ul, const T* ur, int dir, T* fh, const PhysParams& p)
{
    constexpr int NV = Phys2D<EQ>::NV;
    T fl[NV], fr[NV];
    T al, ar;
    if constexpr (EQ == EULER && HLLX) {
        Phys2D<EQ>::flux(ul, dir, fl, p);
        Phys2D<EQ>::flux(ur, dir, fr, p);
        hll_euler<NV, T>(p.flux, dir == 1, ul, ur, fl, fr, Phys2D<EULER>::pressure(ul, p),
                         Phys2D<EULER>::pressure(ur, p), (T)p.gamma, fh);
        return;
    } else if constexpr (EQ == EULER) {
        al = Phys2D<EQ>::flux_speed(ul, dir, fl, p);
        ar = Phys2D<EQ>::flux_speed(ur, dir, fr, p);
    } else {
        Phys2D<EQ>::flux(ul, dir, fl, p);
        Phys2D<EQ>::flux(ur, dir, fr, p);
        al = Phys2D<EQ>::speed(ul, dir, p);
        ar = Phys2D<EQ>::speed(ur, dir, p);
    }
    const T alpha = al > ar ? al : ar;
#pragma unroll
    for (int v = 0; v < NV; ++v) fh[v] = (T)0.5 * (fl[v] + fr[v]) - (T)0.5 * alpha * (ur[v] - ul[v]);
}

// Global index along an axis: wrapped if periodic, -1 if outside.  Callers
// pass indices within a tile and a cell of the domain, so the wrap is a few
// subtractions at most (no 64-bit division).
__device__ __forceinline__ int64_t slot_index(int64_t g, int64_t n, bool periodic)
{
    if (g >= 0 && g < n) return g;
    if (!periodic) return -1;
    while (g < 0) g += n;
    while (g >= n) g -= n;
    return g;
}

__device__ __forceinline__ double shock_line_x(const double x0, const double speed, double y, double t)
{
    return x0 + y * 0.57735026918962576451 + speed * t;  // x0 + y/sqrt(3) + s t
}

// Ghost state for the flux outside side (0 x-lo, 1 x-hi, 2 y-lo, 3 y-hi)
// at the physical point (x, y) and time t.
// Which prescribed state a boundary point sees: 0 none (copy or mirror),
// 1 the Dirichlet state of the side, 2 the post-shock state, 3 the
// pre-shock state; *reflect tells whether the mirror applies.
template <typename TB>
__device__ __forceinline__ int boundary_kind(const Args2D<TB>& a, int side, double x, double y, double t,
                                             bool* reflect)
{
    const int bc = a.bc[side];
    *reflect = bc == BC_REFLECT;
    if (bc == BC_DIRICHLET) return 1;
    if (bc == BC_DMR_WALL) {
        if (x < a.shock_x0) return 2;
        *reflect = true;
        return 0;
    }
    if (bc == BC_DMR_TOP) return x < shock_line_x(a.shock_x0, a.shock_speed, y, t) ? 2 : 3;
    return 0;
}

template <typename TB>
__device__ __forceinline__ double boundary_state(const Args2D<TB>& a, int side, int kind, int v)
{
    // read all three candidates and select the value (a select of their
    // addresses would force the argument block into scratch memory)
    const double d = a.dir[side][v], po = a.post[v], pr = a.pre[v];
    double r = pr;
    r = kind == 2 ? po : r;
    r = kind == 1 ? d : r;
    return r;
}

template <int NV, typename TB, typename T>
__device__ __forceinline__ void ghost_state2d(const Args2D<TB>& a, int side, double x, double y,
                                              double t, const T* in, T* g)
{
    const int dir = side >> 1;
    bool reflect;
    const int kind = boundary_kind(a, side, x, y, t, &reflect);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        if (kind)
            g[v] = (T)boundary_state(a, side, kind, v);
        else if (reflect && v == 1 + dir)
            g[v] = -in[v];
        else
            g[v] = in[v];
    }
}

// |ghost - inner| of the mixed derivative (a1, a2) of variable v at a
// boundary corner at (x, y), from the interior one-sided value `in`.
template <typename TB, typename T>
__device__ __forceinline__ T ghost_jump2d(const Args2D<TB>& a, int side, double x, double y, double t,
                                          int a1, int a2, int v, T in)
{
    const int dir = side >> 1;
    bool reflect;
    const int kind = boundary_kind(a, side, x, y, t, &reflect);
    if (kind) return (a1 == 0 && a2 == 0) ? fabs((T)boundary_state(a, side, kind, v) - in) : fabs(in);
    if (reflect) {
        const int an = dir == 0 ? a1 : a2;
        const bool flip = ((an & 1) != 0) != (v == 1 + dir);  // ghost = -inner
        return flip ? (T)2 * fabs(in) : (T)0;
    }
    return (T)0;
}

__device__ __forceinline__ double combine2(int stage, double un, double adv)
{
    return stage == 0 ? adv : stage == 1 ? 0.75 * un + 0.25 * adv : (1.0 / 3.0) * un + (2.0 / 3.0) * adv;
}
template <typename T>
__device__ __forceinline__ T combine2_t(int stage, T un, T adv)
{
    return stage == 0 ? adv
         : stage == 1 ? (T)0.75 * un + (T)0.25 * adv
                      : (T)(1.0 / 3.0) * un + (T)(2.0 / 3.0) * adv;
}

// P_l^(m)(+-1) as a compile-time constant: side 0 -> -1, side 1 -> +1
__device__ __forceinline__ constexpr double dtr(int l, int m, int side)
{
    return side ? dtrace_r(l, m) : dtrace_l(l, m);
}

// Values of one variable's polynomial at the Q Gauss points of one face
// (FACE 0 left xi=-1, 1 right xi=+1, 2 bottom eta=-1, 3 top eta=+1): first
// the sum across the face, then the along-face Legendre series.  Own cells
// and the tile's ring cells both use this routine, so the two workgroups
// that evaluate a tile-boundary edge flux see bitwise identical traces (the
// FP64 mode-0 update then telescopes exactly).
template <int FACE, int K, typename T>
__device__ __forceinline__ void face_trace_var(const T (&um)[(K + 1) * (K + 1)], T (&tr)[K + 1])
{
    constexpr int K1 = K + 1;
    constexpr bool xface = FACE < 2;
    constexpr bool plus = (FACE & 1) != 0;
    T c[K1];
#pragma unroll
    for (int o = 0; o < K1; ++o) {
        T sum = (T)0;
#pragma unroll
        for (int n = 0; n < K1; ++n) {
            const T val = um[xface ? n * K1 + o : o * K1 + n];
            sum += (plus || !(n & 1)) ? val : -val;
        }
        c[o] = sum;
    }
#pragma unroll
    for (int b = 0; b < K1; ++b) {
        T sum = (T)0;
#pragma unroll
        for (int o = 0; o < K1; ++o) sum += c[o] * (T)leg_at(K1, b, o);
        tr[b] = sum;
    }
}

// Storage plane of mode m = p (k+1) + q: the Q^k space keeps every mode at
// plane m; the P^k space (PK) keeps only the modes p + q <= k, in p-major
// order, and the others are zero by construction.
template <int K, bool PK>
__device__ __forceinline__ constexpr bool mode_kept(int m)
{
    return !PK || m / (K + 1) + m % (K + 1) <= K;
}
template <int K, bool PK>
__device__ __forceinline__ constexpr int mode_plane(int m)
{
    return PK ? (m / (K + 1)) * (K + 1) - (m / (K + 1)) * (m / (K + 1) - 1) / 2 + m % (K + 1) : m;
}

// Modes of variable v of cell c: FP64 mode 0 and the TB modes, all as T
// (the modes the space leaves out as zeros).
template <int K, bool PK, typename TB, typename T>
__device__ __forceinline__ void load_var2d(const StateView<TB>& s, int64_t c, int v, double& m0,
                                           T (&um)[(K + 1) * (K + 1)])
{
    constexpr int NM = (K + 1) * (K + 1);
    m0 = s.m0[v * s.s0 + c];
    um[0] = (T)m0;
#pragma unroll
    for (int m = 1; m < NM; ++m)
        um[m] = mode_kept<K, PK>(m) ? (T)s.hi[v * s.sv + (mode_plane<K, PK>(m) - 1) * s.sl + c] : (T)0;
}

// Value of one variable's polynomial at the cell corner (sx, sy), sx, sy =
// 1 at the +x, +y side: sum_pq u_pq (+-1)^p (+-1)^q, summed in the order p, q
// (P_p(+-1) = (+-1)^p).
template <int K, bool PK, typename T>
__device__ __forceinline__ T corner2d(const T (&u)[(K + 1) * (K + 1)], int sx, int sy)
{
    constexpr int K1 = K + 1;
    T sum = (T)0;
#pragma unroll
    for (int p = 0; p < K1; ++p)
#pragma unroll
        for (int q = 0; q < K1; ++q) {
            if (!mode_kept<K, PK>(p * K1 + q)) continue;
            const bool neg = (!sx && (p & 1)) != (!sy && (q & 1));
            sum += neg ? -u[p * K1 + q] : u[p * K1 + q];
        }
    return sum;
}

// Orders LDS writes before later LDS reads of other lanes of the same
// wavefront (the lanes of one cell always share a wavefront).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Tile of a 1D launch of `ntiles` workgroups over a grid `gx` tiles wide.
// Workgroups are dispatched to the 8 XCDs round-robin by index, and each XCD
// has its own L2; consecutive tile numbers are therefore given to one XCD.
// Tiles are numbered in strips of 32 tile columns, row by row inside a strip
// (the last strip as wide as what is left), so the tile above a tile was
// processed one strip row earlier on the same XCD: the neighbour rows and
// columns a tile reads are still in that L2.
__device__ __forceinline__ void xcd_tile(int64_t gx, int64_t ntiles, int64_t& bx, int64_t& by)
{
    // tile counts stay far below 2^32 (a launch has at most 2^32 - 1 workgroups)
    constexpr uint32_t W = 32;
    const uint32_t p = blockIdx.x, q = (uint32_t)ntiles >> 3, r = (uint32_t)ntiles & 7;
    const uint32_t x = p & 7, k = p >> 3;
    const uint32_t l = x * q + (x < r ? x : r) + k;
    const uint32_t ux = (uint32_t)gx, uy = (uint32_t)ntiles / ux;
    const uint32_t full = ux / W, in_full = full * W * uy;
    if (l < in_full) {
        const uint32_t st = l / (W * uy), w = l % (W * uy);
        bx = st * W + w % W;
        by = w / W;
    } else {
        const uint32_t rest = ux - full * W, w = l - in_full;
        bx = full * W + w % rest;
        by = w / rest;
    }
}

// Split of a gx x gy tile grid into the interior tiles [x0, x1) x [y0, y1),
// none of whose cells has a face on a non-periodic domain edge, and the
// boundary tiles around them (all others).
struct TileSplit {
    int64_t gx, gy, x0, x1, y0, y1;
    int64_t interior() const { return (x1 - x0) * (y1 - y0); }
    int64_t boundary() const { return gx * gy - interior(); }
};

// Boundary tile i of a split: first the rows outside [y0, y1) over the full
// width, then the columns outside [x0, x1) over the rows inside.
__device__ __forceinline__ void ring_tile(uint32_t i, const TileSplit& t, int64_t& bx, int64_t& by)
{
    const uint32_t gx = (uint32_t)t.gx, lo_rows = (uint32_t)t.y0;
    const uint32_t row_tiles = (uint32_t)(t.gy - (t.y1 - t.y0)) * gx;
    if (i < row_tiles) {
        const uint32_t r = i / gx;
        bx = i % gx;
        by = r < lo_rows ? r : t.y1 + (r - lo_rows);
    } else {
        const uint32_t lo_cols = (uint32_t)t.x0, ncols = (uint32_t)(t.gx - (t.x1 - t.x0));
        const uint32_t j = i - row_tiles, c = j % ncols;
        by = t.y0 + j / ncols;
        bx = c < lo_cols ? c : t.x1 + (c - lo_cols);
    }
}

// ---------------------------------------------------------------------------
// Positivity-preserving limiter on rectangles (Zhang and Shu), applied after
// the jump filter / hybrid limiter (the paper's Sec. 3.2 examples with
// extreme positivity demands).  Test points: (Gauss-Lobatto x Gauss) and
// (Gauss x Gauss-Lobatto) with N = ceil((k+3)/2) Lobatto points (the Q^k
// cell average is a convex combination of the values at the first set, and
// the sets contain the edge Gauss points of the fluxes), then the Gauss x
// Gauss points of the volume quadrature.
template <int K>
struct PP2DPoints {
    static constexpr int Q = K + 1;
    static constexpr int N = (K + 4) / 2 < 2 ? 2 : (K + 4) / 2;
    static constexpr int NP = 2 * N * Q + Q * Q;
};

// P_l at Lobatto node i: 0 -> -1, 1 -> +1, 2 -> 0.
__device__ __forceinline__ constexpr double lob_leg(int i, int l)
{
    return i == 0 ? ((l & 1) ? -1.0 : 1.0) : i == 1 ? 1.0 : (l == 0 ? 1.0 : l == 2 ? -0.5 : 0.0);
}

// P_p(xi) (dir 0) or P_q(eta) (dir 1) at test point i.
template <int K>
__device__ __forceinline__ constexpr double pp2_leg(int i, int dir, int l)
{
    constexpr int Q = PP2DPoints<K>::Q, N = PP2DPoints<K>::N;
    if (i < 2 * N * Q) {
        const int set = i / (N * Q), r = i % (N * Q), lob = r / Q, g = r % Q;
        return (set == dir) ? lob_leg(lob, l) : leg_at(Q, g, l);
    }
    const int r = i - 2 * N * Q;
    return leg_at(Q, dir == 0 ? r / Q : r % Q, l);
}

__device__ __forceinline__ double pp2_pressure(double gamma, const double (&w)[4])
{
    return (gamma - 1.0) * (w[3] - 0.5 * (w[1] * w[1] + w[2] * w[2]) / w[0]);
}

// True when the limiter provably leaves the cell unchanged: |P_p P_q| <= 1
// on the cell, so rho_bar - sum |rho_pq| bounds the density and (gamma - 1)
// (E_lo - (Mx_hi^2 + My_hi^2) / (2 rho_lo)) the pressure from below at every
// point; both must exceed twice the largest threshold and rounding margin the
// limiter could apply (as in the 1D screen).  ubar[v], sabs[v] = sum over the
// modes >= 1 of |u_m| (FP64).
template <typename TB>
__device__ __forceinline__ bool pp2_clear(const double (&ubar)[4], const double (&sabs)[4], double gamma)
{
    constexpr double ur = sizeof(TB) == 4 ? 0x1p-23 : 0x1p-52;
    const double rlo = ubar[0] - sabs[0], sr = fabs(ubar[0]) + sabs[0];
    if (!(rlo > 2.0 * (1e-13 + 8.0 * ur * sr))) return false;
    const double mx = fabs(ubar[1]) + sabs[1], my = fabs(ubar[2]) + sabs[2];
    const double elo = ubar[3] - sabs[3], se = fabs(ubar[3]) + sabs[3];
    // (1/rlo by the reciprocal helper: the margins below are two-fold)
    const double irlo = trcp<double>(rlo);
    const double kin = 0.5 * (mx * mx + my * my) * irlo;
    const double plo = (gamma - 1.0) * (elo - kin);
    const double mmax = 8.0 * ur * (se + 2.0 * kin + kin * sr * irlo);
    return plo > 2.0 * (1e-13 + mmax);
}

__device__ __forceinline__ double wave_min(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(v, off, 64);
        v = (o < v || o != o) ? o : v;
    }
    return v;
}

// Point value at test point i of the cell whose coefficients (FP64 average,
// then the modes >= 1 as stored) are in c[v * NM + m], and the sums of the
// magnitudes of its terms.
template <int K, bool PK>
__device__ __forceinline__ void pp2_point_lds(const double* c, int i, double (&w)[4], double (&wa)[4])
{
    constexpr int K1 = K + 1, NM = K1 * K1;
    double px[K1], py[K1];
#pragma unroll
    for (int l = 0; l < K1; ++l) {
        px[l] = pp2_leg<K>(i, 0, l);
        py[l] = pp2_leg<K>(i, 1, l);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        double sum = c[v * NM], sa = fabs(c[v * NM]);
#pragma unroll
        for (int m = 1; m < NM; ++m) {
            if (!mode_kept<K, PK>(m)) continue;
            const double t = (c[v * NM + m] * px[m / K1]) * py[m % K1];
            sum += t;
            sa += fabs(t);
        }
        w[v] = sum;
        wa[v] = sa;
    }
}

// Positivity limiter of one cell by one wavefront.  Lane l < 4 NM holds
// coefficient l = v NM + m in `cf` (the FP64 average for m = 0, a mode
// rounded to TB otherwise) and the wave's LDS block c mirrors them; lane
// i < NP takes test point i.  The steps are those of the 1D limiter on the
// 2D test points: the density's modes >= 1 scaled so the density at every
// point is >= eps_r, then all modes >= 1 so the pressure is >= eps_p (60
// bisection steps on the segment from the average to each point value,
// along which the pressure is concave), eps = min(1e-13, rho_bar, p_bar)
// raised per point to the rounding margin of its value (8 units of
// roundoff of the modes' precision times the magnitudes that cancel), which
// vanishes in exact arithmetic; finally the cell is checked in the fluxes'
// own arithmetic (precision TB, pressure as the flux computes it) and its
// modes >= 1 halved until density and pressure are positive at every point
// (dropped after 50 halvings).  Minima over the points are taken across the
// lanes.  The averages never change.  Returns true when the cell changed;
// sets *reject (nullable) when its average is inadmissible.
template <int K, bool PK, typename TB>
__device__ __forceinline__ bool pp2_wave(double* c, double& cf, int lane, double gamma, int* reject)
{
    constexpr int K1 = K + 1, NM = K1 * K1, NC = 4 * NM, NP = PP2DPoints<K>::NP;
    constexpr double ur = sizeof(TB) == 4 ? 0x1p-23 : 0x1p-52;
    static_assert(NP <= 64 && NC <= 64, "one lane per test point and per coefficient");
    const int m = lane % NM;
    const bool coef = lane < NC && m > 0;
    if (lane < NC) c[lane] = cf;
    wave_lds_sync();
    double ub[4], sabs[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        ub[v] = c[v * NM];
        double t = 0.0;
#pragma unroll
        for (int q = 1; q < NM; ++q) t += fabs(c[v * NM + q]);
        sabs[v] = t;
    }
    if (pp2_clear<TB>(ub, sabs, gamma)) return false;
    const double pb = pp2_pressure(gamma, ub);
    if (!(ub[0] > 0.0) || !(pb > 0.0)) {
        if (lane == 0 && reject) atomicOr(reject, 1);
        return false;
    }
    double eps = 1e-13;
    if (ub[0] < eps) eps = ub[0];
    if (pb < eps) eps = pb;
    const bool pt = lane < NP;
    // density
    {
        double w[4], wa[4];
        pp2_point_lds<K, PK>(c, pt ? lane : 0, w, wa);
        const double rmin = wave_min(pt ? w[0] : INFINITY);
        double eps_r = wave_max(pt ? 8.0 * ur * wa[0] : 0.0);
        if (eps_r < eps) eps_r = eps;
        if (eps_r > ub[0]) eps_r = ub[0];
        if (rmin < eps_r) {
            double th = (ub[0] - eps_r) / (ub[0] - rmin);
            if (th < 0.0) th = 0.0;
            wave_lds_sync();
            if (coef && lane < NM) {
                cf = (double)(TB)(cf * th);
                c[lane] = cf;
            }
            wave_lds_sync();
        }
    }
    // pressure
    {
        double t = 1.0;
        if (pt) {
            double w[4], wa[4];
            pp2_point_lds<K, PK>(c, lane, w, wa);
            double eps_i = eps;
            if (w[0] > 0.0) {
                const double kin = 0.5 * (w[1] * w[1] + w[2] * w[2]) / w[0];
                const double mg = 8.0 * ur * (wa[3] + (fabs(w[1]) * wa[1] + fabs(w[2]) * wa[2]) / w[0] +
                                              kin * wa[0] / w[0]);
                if (mg > eps_i) eps_i = mg;
            }
            if (eps_i > pb) eps_i = pb;
            if (!(pp2_pressure(gamma, w) >= eps_i)) {
                double lo = 0.0, hi = 1.0;
                for (int it = 0; it < 60; ++it) {
                    const double mid = 0.5 * (lo + hi);
                    double wm[4];
#pragma unroll
                    for (int v = 0; v < 4; ++v) wm[v] = ub[v] + mid * (w[v] - ub[v]);
                    if (pp2_pressure(gamma, wm) >= eps_i)
                        lo = mid;
                    else
                        hi = mid;
                }
                t = lo;
            }
        }
        const double theta = wave_min(t);
        if (theta < 1.0) {
            wave_lds_sync();
            if (coef) {
                cf = (double)(TB)(cf * theta);
                c[lane] = cf;
            }
            wave_lds_sync();
        }
    }
    // positivity in the fluxes' own arithmetic
    for (int halving = 0; halving <= 50; ++halving) {
        bool ok = true;
        if (pt) {
            TB w[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                TB sum = (TB)c[v * NM];
#pragma unroll
                for (int q = 1; q < NM; ++q)
                    if (mode_kept<K, PK>(q))
                        sum += (TB)c[v * NM + q] *
                               (TB)(pp2_leg<K>(lane, 0, q / K1) * pp2_leg<K>(lane, 1, q % K1));
                w[v] = sum;
            }
            const TB ir = (TB)1 / w[0];
            const TB pr = ((TB)gamma - (TB)1) * (w[3] - (TB)0.5 * (w[1] * (w[1] * ir) + w[2] * (w[2] * ir)));
            ok = w[0] > (TB)0 && pr > (TB)0;
        }
        if (__ballot(!ok) == 0) break;
        const double f = halving < 50 ? 0.5 : 0.0;
        wave_lds_sync();
        if (coef) {
            cf = (double)((TB)cf * (TB)f);
            c[lane] = cf;
        }
        wave_lds_sync();
    }
    return true;
}

// Screen of a cell held by NV = 4 adjacent lanes (lane v holds variable v:
// FP64 average m0 and the sum of |modes >= 1|); true in every lane of the
// cell when the limiter would leave it unchanged.
template <typename TB>
__device__ __forceinline__ bool pp2_clear_lanes(double m0, double sabs, int base, double gamma)
{
    double ub[4], sa[4];
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        ub[w] = __shfl(m0, base + w, 64);
        sa[w] = __shfl(sabs, base + w, 64);
    }
    return pp2_clear<TB>(ub, sa, gamma);
}

}  // namespace

// -------------------------------------------------------------------------
// Residual + Shu-Osher combination (no filter) -> a.out.  With alpha_acc the
// kernel accumulates the CFL quantity max(lambda_x/hx + lambda_y/hy) of its
// output's cell averages.
// Mapping: one lane per (cell, variable), the NV lanes of a cell adjacent;
// FX x FY cells per workgroup (16 x 4 for Euler).  Each lane evaluates its
// variable's traces and point values; whole states at a point are gathered
// inside the cell's lane group (a rotation transpose of shuffles), so every
// flux is evaluated once: edge fluxes by (edge, point) work items over the
// whole workgroup, volume fluxes with the NV lanes of a cell taking one
// Gauss point of the current row each.
// -------------------------------------------------------------------------
template <int NV>
struct StageTile {
    static constexpr int FX = 16, FY = 256 / (16 * NV);
    static constexpr int NVE = FY * (FX + 1);  // vertical edges (x = const)
    static constexpr int NHE = FX * (FY + 1);  // horizontal edges
};

template <int EQ, int K, typename TB, bool PK, bool HLLX>
__global__ __launch_bounds__(256) void stage2d_kernel(Args2D<TB> a)
{
    using P = Phys2D<EQ>;
    using T = TB;
    constexpr int NV = P::NV, K1 = K + 1, NM = K1 * K1, Q = K1;
    constexpr int FX = StageTile<NV>::FX, FY = StageTile<NV>::FY;
    constexpr int NVE = StageTile<NV>::NVE, NHE = StageTile<NV>::NHE;
    // One edge holds Q points x NV variables in ES words, entry (b, v) at
    // sw(b, v); the exchange block of a cell holds NV x NV entries in XS
    // words, entry (i, j) at sw(i, j).  With 4 variables the entries are
    // rotated, sw(i, j) = 4 i + (i + j) mod 4, and ES, XS are odd multiples
    // of 4 words (4 or 12 mod 16): then each group of 16 lanes (4 cells x 4
    // variables, one 128-byte LDS cycle of 64-bit accesses) hits 16
    // different banks whether the lanes vary the cell and the variable
    // (traces, edge fluxes per cell, point values) or the edge and the point
    // (the flux work items; with Q = 3 two of them share a bank).  ES is the
    // smallest such stride that holds the 4 Q words, which keeps the tile's
    // LDS for Q <= 3 low enough for a fourth workgroup per CU.
    constexpr int ES = NV == 4 ? 4 * (Q | 1) : Q + 1;
    constexpr int XS = NV == 4 ? 20 : 1;
    auto sw = [](int i, int j) { return NV == 4 ? 4 * i + ((i + j) & 3) : i * NV + j; };
    // traces: lower side (the -x / -y cell) and upper side of every edge
    // (vertical edges first); the lower half later takes the edge fluxes and
    // the upper half the per-cell exchange blocks of the volume term (NV x NV
    // values per cell: point values, then F1, then F2)
    constexpr int HALF = (NVE + NHE) * ES;
    constexpr int XB = NV > 1 ? (256 / NV) * XS : 0;
    __shared__ __align__(16) T lds[HALF + (HALF > XB ? HALF : XB)];
    T* sLo = lds;
    T* sHi = lds + HALF;
    T* sF = lds;
    T* sX = lds + HALF;

    // the positivity limiter's list of this stage starts empty (the kernels
    // that append to it and read it run after this one)
    if (a.pcount && blockIdx.x == 0 && threadIdx.x == 0) *a.pcount = 0;
    if (a.dt_from_ctrl && a.ctrl->done) return;
    const double dt = a.dt_from_ctrl ? a.ctrl->dt : a.dt_host;
    const double t0 = a.dt_from_ctrl ? a.ctrl->t : a.t_host;
    const int stage = a.stage;
    const double ts = t0 + (stage == 0 ? 0.0 : stage == 1 ? dt : 0.5 * dt);

    const int tid = threadIdx.x, v = tid % NV, cidx = tid / NV, base = tid - v;
    const int tx = cidx % FX, ty = cidx / FX;
    int64_t tbx, tby;
    xcd_tile((a.nx + FX - 1) / FX, gridDim.x, tbx, tby);
    const int64_t ix0 = tbx * FX, jy0 = tby * FY;
    const int64_t ix = ix0 + tx, jy = jy0 + ty;
    const bool px = a.bc[0] == BC_PERIODIC, py = a.bc[2] == BC_PERIODIC;
    const int64_t cx = slot_index(ix, a.nx, px), cy = slot_index(jy, a.ny, py);
    const bool loadable = cx >= 0 && cy >= 0;
    const bool own = ix < a.nx && jy < a.ny;
    // edge slots: vertical edge e (0..FX) of row r -> r*(FX+1)+e;
    // horizontal edge e (0..FY) of column c -> NVE + c*(FY+1)+e
    auto vslot = [&](int r, int e) { return r * (FX + 1) + e; };
    auto hslot = [&](int c, int e) { return NVE + c * (FY + 1) + e; };

    // ---- phase 1: own traces (and the ring's facing traces) to LDS ----
    // The own modes and the ring cell's modes are requested together, so the
    // two trips to memory overlap.
    double m0v = 0.0;
    T um[NM];
#pragma unroll
    for (int m = 0; m < NM; ++m) um[m] = (T)0;
    if (loadable) load_var2d<K, PK, TB, T>(a.us, cy * a.nx + cx, v, m0v, um);
    const int64_t cell = jy * a.nx + ix;
    constexpr int NRING = 2 * FY + 2 * FX;
    const int r = tid / NV, rv = tid % NV;
    int g = 0, i = 0;  // g: 0 left column, 1 right column, 2 bottom row, 3 top row
    if (r < FY) { g = 0; i = r; }
    else if (r < 2 * FY) { g = 1; i = r - FY; }
    else if (r < 2 * FY + FX) { g = 2; i = r - 2 * FY; }
    else { g = 3; i = r - 2 * FY - FX; }
    bool ring = false;
    T wm[NM];
#pragma unroll
    for (int m = 0; m < NM; ++m) wm[m] = (T)0;
    if (tid < NRING * NV) {
        const int64_t gx = g == 0 ? ix0 - 1 : g == 1 ? ix0 + FX : ix0 + i;
        const int64_t gy = g == 2 ? jy0 - 1 : g == 3 ? jy0 + FY : jy0 + i;
        const int64_t hx_ = slot_index(gx, a.nx, px), hy_ = slot_index(gy, a.ny, py);
        ring = hx_ >= 0 && hy_ >= 0;
        if (ring) {
            double w0;
            load_var2d<K, PK, TB, T>(a.us, hy_ * a.nx + hx_, rv, w0, wm);
        }
    }
    if (loadable) {
        T tr[Q];
        face_trace_var<0, K, T>(um, tr);  // left face: upper side of vertical edge tx
#pragma unroll
        for (int b = 0; b < Q; ++b) sHi[vslot(ty, tx) * ES + sw(b, v)] = tr[b];
        face_trace_var<1, K, T>(um, tr);  // right face: lower side of edge tx+1
#pragma unroll
        for (int b = 0; b < Q; ++b) sLo[vslot(ty, tx + 1) * ES + sw(b, v)] = tr[b];
        face_trace_var<2, K, T>(um, tr);  // bottom face: upper side of horizontal edge ty
#pragma unroll
        for (int b = 0; b < Q; ++b) sHi[hslot(tx, ty) * ES + sw(b, v)] = tr[b];
        face_trace_var<3, K, T>(um, tr);  // top face: lower side of edge ty+1
#pragma unroll
        for (int b = 0; b < Q; ++b) sLo[hslot(tx, ty + 1) * ES + sw(b, v)] = tr[b];
    }
    if (ring) {
        T tr[Q];
        T* dst;
        if (g == 0) {
            face_trace_var<1, K, T>(wm, tr);
            dst = &sLo[vslot(i, 0) * ES];
        } else if (g == 1) {
            face_trace_var<0, K, T>(wm, tr);
            dst = &sHi[vslot(i, FX) * ES];
        } else if (g == 2) {
            face_trace_var<3, K, T>(wm, tr);
            dst = &sLo[hslot(i, 0) * ES];
        } else {
            face_trace_var<2, K, T>(wm, tr);
            dst = &sHi[hslot(i, FY) * ES];
        }
#pragma unroll
        for (int b = 0; b < Q; ++b) dst[sw(b, rv)] = tr[b];
    }
    __syncthreads();

    // u^n of the own cell (stages 2 and 3).  FP64: requested now, so that its
    // trip to memory overlaps the flux and volume phases, and folded into
    // the accumulators at the start of phase 3 (no registers of its own in
    // the volume loop, which sets the register count); FP32 (mixed) modes
    // keep the plain combination at the end, where the fold's larger
    // intermediate would cost precision, and so do the HLL/HLLC kernels,
    // whose flux phase has no registers to spare.
    constexpr bool FOLD = sizeof(T) == 8 && !HLLX;
    double n0 = 0.0;
    T nm[NM];
#pragma unroll
    for (int m = 0; m < NM; ++m) nm[m] = (T)0;
    if (FOLD && own && stage > 0) load_var2d<K, PK, TB, T>(a.un, cell, v, n0, nm);

    // ---- phase 2: LLF flux at every (edge, Gauss point) of the tile ----
    constexpr int NITEM = (NVE + NHE) * Q;
    constexpr int PER = (NITEM + 255) / 256;
    // Each (edge, point) item is the only reader of its lower-side trace
    // entries, so it overwrites them with its flux at once: no other lane
    // reads that slot, and the flux needs no registers until a barrier.
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int w = tid + 256 * k;
        if (w >= NITEM) break;
        const int es = w / Q, b = w % Q;
        const bool vert = es < NVE;
        int64_t glo, ghi;  // global coordinates of the lower and upper cells
        int64_t other;     // the cell coordinate along the edge
        if (vert) {
            const int r = es / (FX + 1), e = es % (FX + 1);
            glo = ix0 + e - 1;
            ghi = ix0 + e;
            other = jy0 + r;
        } else {
            const int c = (es - NVE) / (FY + 1), e = (es - NVE) % (FY + 1);
            glo = jy0 + e - 1;
            ghi = jy0 + e;
            other = ix0 + c;
        }
        const int64_t nax = vert ? a.nx : a.ny, nal = vert ? a.ny : a.nx;
        const bool per = vert ? px : py, per_o = vert ? py : px;
        const bool lo_ok = slot_index(glo, nax, per) >= 0, hi_ok = slot_index(ghi, nax, per) >= 0;
        const bool o_ok = slot_index(other, nal, per_o) >= 0;
        T f[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) f[q] = (T)0;
        if (o_ok && (lo_ok || hi_ok)) {
            T ul[NV], ur[NV];
#pragma unroll
            for (int q = 0; q < NV; ++q) {
                ul[q] = sLo[es * ES + sw(b, q)];
                ur[q] = sHi[es * ES + sw(b, q)];
            }
            const double edge = vert ? a.xlo + (double)ghi * a.hx : a.ylo + (double)ghi * a.hy;
            const double along = vert ? a.ylo + (double)other * a.hy + 0.5 * a.hy * (1.0 + gl_node(Q, b))
                                      : a.xlo + (double)other * a.hx + 0.5 * a.hx * (1.0 + gl_node(Q, b));
            const double xq = vert ? edge : along, yq = vert ? along : edge;
            if (!lo_ok) ghost_state2d<NV, TB, T>(a, vert ? 0 : 2, xq, yq, ts, ur, ul);
            if (!hi_ok) ghost_state2d<NV, TB, T>(a, vert ? 1 : 3, xq, yq, ts, ul, ur);
            llf2d<EQ, T, HLLX>(ul, ur, vert ? 0 : 1, f, a.phys);
        }
#pragma unroll
        for (int q = 0; q < NV; ++q) sF[es * ES + sw(b, q)] = f[q];
    }
    __syncthreads();  // fluxes complete; the upper half takes the exchange blocks

    // ---- phase 3: volume term, edge terms, combination (variable v) ----
    const T hy2 = (T)(0.5 * a.hy), hx2 = (T)(0.5 * a.hx);
    T acc[NM];
#pragma unroll
    for (int m = 0; m < NM; ++m) acc[m] = (T)0;
    if constexpr (FOLD) {
        // out = c0 u^n + c1 (u + dt L) = c1 (u + dt L'), L' = L + (c0/c1) u^n /
        // dt: with L = (2p+1)(2q+1)/(hx hy) r, r seeded with
        // (c0/c1) u^n hy hx / ((2p+1)(2q+1) dt); c0/c1 = 3 (stage 2), 1/2 (stage 3)
        // (dt = 0, a per-call stage: dt L vanishes, so u^n is added to u
        // instead, which the volume term no longer needs)
        if (stage > 0) {
            const double ratio = stage == 1 ? 3.0 : 0.5;
            const double base = ratio * a.hx * a.hy / dt;
#pragma unroll
            for (int p = 0; p < K1; ++p)
#pragma unroll
                for (int q = 0; q < K1; ++q) {
                    const int m = p * K1 + q;
                    if (m == 0 || !mode_kept<K, PK>(m)) continue;
                    if (dt != 0.0)
                        acc[m] = nm[m] * (T)(base * (1.0 / (double)((2 * p + 1) * (2 * q + 1))));
                    else
                        um[m] = um[m] + (T)ratio * nm[m];
                }
        }
    }
    // Volume term: (hy/2) sum w_a w_b F1 P_p'(xi_a) P_q(eta_b)
    //            + (hx/2) sum w_a w_b F2 P_p(xi_a) P_q'(eta_b)
#pragma unroll
    for (int qa = 0; qa < Q; ++qa) {
        T col[K1];  // sum_p u^{pq} P_p(xi_a)
#pragma unroll
        for (int q = 0; q < K1; ++q) {
            T sum = (T)0;
#pragma unroll
            for (int p = 0; p < K1; ++p) sum += um[p * K1 + q] * (T)leg_at(Q, qa, p);
            col[q] = sum;
        }
        constexpr int NB = NV > Q ? NV : Q;
        T uv[NB];  // this variable at the points (qa, b)
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            T sum = (T)0;
            if (b < Q) {
#pragma unroll
                for (int q = 0; q < K1; ++q) sum += col[q] * (T)leg_at(Q, (b < Q ? b : 0), q);
            }
            uv[b] = sum;
        }
        T g1[NB], g2[NB];  // F1, F2 of this variable at the points (qa, b)
        if constexpr (NV == 1) {
            // scalar equations: the lane evaluates every point itself
#pragma unroll
            for (int b = 0; b < Q; ++b) {
                T u1[1] = {uv[b]}, h1[1], h2[1];
                P::flux(u1, 0, h1, a.phys);
                P::flux(u1, 1, h2, a.phys);
                g1[b] = h1[0];
                g2[b] = h2[0];
            }
        } else {
            // lane v of the cell takes point (qa, v): the cell's lanes swap
            // point values and fluxes through their LDS block
            T* X = &sX[cidx * XS];
#pragma unroll
            for (int b = 0; b < NV; ++b) X[sw(b, v)] = uv[b];
            wave_lds_sync();
            T uq[NV], f1[NV], f2[NV];
#pragma unroll
            for (int q = 0; q < NV; ++q) {
                uq[q] = X[sw(v, q)];
                f1[q] = f2[q] = (T)0;
            }
            wave_lds_sync();  // the block is rewritten with F1
            if (v < Q && own) {
                if (EQ == EULER && a.check) {
                    // the flux's own reciprocal of the density (shared with it)
                    const T ir = trcp<T>(uq[0]);
                    const T pr = ((T)a.phys.gamma - (T)1) *
                                 (uq[3] - (T)0.5 * (uq[1] * (uq[1] * ir) + uq[2] * (uq[2] * ir)));
                    if (!(uq[0] > (T)0) || !(pr > (T)0)) {
                        const bool fin = isfinite((double)uq[0]) && isfinite((double)pr);
                        latch_error(a.ctrl, fin ? -5 : -4, cell);
                    }
                }
                P::flux(uq, 0, f1, a.phys);
                P::flux(uq, 1, f2, a.phys);
            }
#pragma unroll
            for (int q = 0; q < NV; ++q) X[sw(v, q)] = f1[q];
            wave_lds_sync();
#pragma unroll
            for (int b = 0; b < NB; ++b) g1[b] = X[sw(b, v)];
            wave_lds_sync();  // then with F2
#pragma unroll
            for (int q = 0; q < NV; ++q) X[sw(v, q)] = f2[q];
            wave_lds_sync();
#pragma unroll
            for (int b = 0; b < NB; ++b) g2[b] = X[sw(b, v)];
            wave_lds_sync();  // the block is rewritten by the next row
        }
        // t1[q] = wa hy/2 sum_b w_b F1 P_q(eta_b), t2[q] = wa hx/2 sum_b w_b
        // F2 P_q'(eta_b); P_0' = 0, so t2[0] and the p = 0 terms of F1 vanish
        // and are not formed
        T t1[K1], t2[K1];
#pragma unroll
        for (int q = 0; q < K1; ++q) t1[q] = t2[q] = (T)0;
#pragma unroll
        for (int b = 0; b < Q; ++b) {
            const T w1 = (T)gl_weight(Q, b) * g1[b], w2 = (T)gl_weight(Q, b) * g2[b];
#pragma unroll
            for (int q = 0; q < K1; ++q) {
                t1[q] += w1 * (T)leg_at(Q, b, q);
                if (q > 0) t2[q] += w2 * (T)dleg_at(Q, b, q);
            }
        }
        const T s1 = (T)gl_weight(Q, qa) * hy2, s2 = (T)gl_weight(Q, qa) * hx2;
#pragma unroll
        for (int q = 0; q < K1; ++q) {
            t1[q] *= s1;
            t2[q] *= s2;
        }
#pragma unroll
        for (int p = 0; p < K1; ++p)
#pragma unroll
            for (int q = 0; q < K1; ++q) {
                if ((p == 0 && q == 0) || !mode_kept<K, PK>(p * K1 + q)) continue;
                T r = acc[p * K1 + q];
                if (p > 0) r += (T)dleg_at(Q, qa, p) * t1[q];
                if (q > 0) r += (T)leg_at(Q, qa, p) * t2[q];
                acc[p * K1 + q] = r;
            }
        // keep the rows apart: interleaving them only raises the register
        // count (and so lowers the occupancy)
        __builtin_amdgcn_sched_barrier(0);
    }

    double v0 = 0.0;
    if (own) {
        const T* FL = &sF[vslot(ty, tx) * ES];
        const T* FR = &sF[vslot(ty, tx + 1) * ES];
        const T* FB = &sF[hslot(tx, ty) * ES];
        const T* FT = &sF[hslot(tx, ty + 1) * ES];
        const double ivol = a.inv_hx * a.inv_hy;
        // mode (0,0): -(hy/2) sum_b w_b (FR - FL) - (hx/2) sum_a w_a (FT - FB), in FP64
        double ex = 0.0, ey = 0.0;
#pragma unroll
        for (int b = 0; b < Q; ++b) {
            ex += gl_weight(Q, b) * ((double)FR[sw(b, v)] - (double)FL[sw(b, v)]);
            ey += gl_weight(Q, b) * ((double)FT[sw(b, v)] - (double)FB[sw(b, v)]);
        }
        const double L0 = -(0.5 * a.hy * ex + 0.5 * a.hx * ey) * ivol;
        // modes >= 1: the edge moments of each face, sum_b w_b F_b P_o(b),
        // enter mode (p, q) with the sign (-1)^p (left) or (-1)^q (bottom) of
        // P_p(-1), P_q(-1); L overwrites acc
        {
            T xr[K1], xl[K1], yt[K1], yb[K1];
#pragma unroll
            for (int o = 0; o < K1; ++o) xr[o] = xl[o] = yt[o] = yb[o] = (T)0;
#pragma unroll
            for (int b = 0; b < Q; ++b) {
                const T wr = (T)gl_weight(Q, b) * FR[sw(b, v)], wl = (T)gl_weight(Q, b) * FL[sw(b, v)];
                const T wt = (T)gl_weight(Q, b) * FT[sw(b, v)], wb = (T)gl_weight(Q, b) * FB[sw(b, v)];
#pragma unroll
                for (int o = 0; o < K1; ++o) {
                    const T lb = (T)leg_at(Q, b, o);
                    xr[o] += wr * lb;
                    xl[o] += wl * lb;
                    yt[o] += wt * lb;
                    yb[o] += wb * lb;
                }
            }
#pragma unroll
            for (int p = 0; p < K1; ++p)
#pragma unroll
                for (int q = 0; q < K1; ++q) {
                    if ((p == 0 && q == 0) || (PK && p + q > K)) continue;
                    const T ex_ = (p & 1) ? xr[q] + xl[q] : xr[q] - xl[q];
                    const T ey_ = (q & 1) ? yt[p] + yb[p] : yt[p] - yb[p];
                    const T r = acc[p * K1 + q] - hy2 * ex_ - hx2 * ey_;
                    acc[p * K1 + q] = (T)((2 * p + 1) * (2 * q + 1)) * (T)ivol * r;
                }
        }
        // Euler step u + dt L in place, pinned (empty asm) before the loads of
        // u^n so that they do not hold registers during the flux sums
        double w0 = m0v + dt * L0;
        asm volatile("" : "+v"(w0));
#pragma unroll
        for (int m = 1; m < NM; ++m) {
            if (!mode_kept<K, PK>(m)) continue;
            um[m] = um[m] + (T)dt * acc[m];
            asm volatile("" : "+v"(um[m]));
        }
        asm volatile("" ::: "memory");
        // u^n of the own cell for the combination (FP64: loaded early, its
        // modes >= 1 already in um through the fold)
        if (!FOLD && stage > 0) load_var2d<K, PK, TB, T>(a.un, cell, v, n0, nm);
        v0 = combine2(stage, n0, w0);
        a.out.m0[v * a.out.s0 + cell] = v0;
#pragma unroll
        for (int m = 1; m < NM; ++m) {
            if (!mode_kept<K, PK>(m)) continue;
            um[m] = combine2_t<T>(stage, FOLD ? (T)0 : nm[m], um[m]);
            a.out.hi[v * a.out.sv + (mode_plane<K, PK>(m) - 1) * a.out.sl + cell] = um[m];
        }
        if (a.corner) {
            // the output's values at the cell corners, for the hybrid
            // indicator: the same sums over the stored modes that the
            // indicator forms from the state (corner2d)
            um[0] = (T)v0;
#pragma unroll
            for (int c = 0; c < 4; ++c)
                a.corner[(c * NV + v) * a.cstride + cell] = corner2d<K, PK, T>(um, c & 1, c >> 1);
            if constexpr (EQ == EULER) {
                if (a.ppfail) {
                    double sabs = 0.0;
#pragma unroll
                    for (int m = 1; m < NM; ++m)
                        if (mode_kept<K, PK>(m)) sabs += fabs((double)um[m]);
                    const bool clear = pp2_clear_lanes<TB>(v0, sabs, base, a.phys.gamma);
                    if (v == 0) a.ppfail[cell] = clear ? 0 : 1;
                }
            }
        }
    }
    // CFL quantity of the output's cell average (all variables of the cell)
    if (a.alpha_acc) {
        double w0[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) w0[q] = NV > 1 ? __shfl(v0, base + q, 64) : v0;
        const double lam = own ? P::cfl(w0, a.inv_hx, a.inv_hy, a.phys) : 0.0;
        const double z = wave_max(lam);
        if ((tid & 63) == 0) atomic_max_nonneg(a.alpha_acc, z);
    }
}

// -------------------------------------------------------------------------
// Jump filter: filtered copy of a.us into a.out, then (pp) the positivity
// limiter's screen (the hybrid limiter has kernels of its own below).
//   E^l = dt / (hx hy H) * max_v [cfmx beta_x Sx^l_v + cfmy beta_y Sy^l_v],
//   Sx^l = sum_{|a| <= l} jsx[a] * Jx^a (edge-averaged |[d^a u]| in reference
//   derivatives; jsx[0] = hx, jsx[a] = m(m+1) hx^(m+1) (2/hx)^a1 (2/hy)^a2).
// Mapping: one lane per (cell, variable); the NV lanes of a cell are
// adjacent, so the maximum over the variables is a reduction inside a group
// of NV lanes.  A workgroup covers FX x FY cells (16 x 4 for Euler) and
// stages their modes and those of the four face-neighbour rows/columns in
// LDS; each lane keeps only its own variable's modes in registers.
// -------------------------------------------------------------------------
template <int NV>
struct FilterTile {
    static constexpr int FX = 16, FY = 256 / (16 * NV);
    static constexpr int SX = FX + 2, SY = FY + 2;
};

// BND: the launch over the boundary tiles of the split, with the ghost
// jumps of faces on the domain edge; without it, the launch over the
// interior tiles, whose faces all have a neighbour cell (that code holds no
// registers for the boundary cases: 124 instead of 163 VGPRs for FP64 Q^2).
template <int EQ, int K, typename TB, bool PK, bool BND>
__global__ __launch_bounds__(256) void filter2d_kernel(Args2D<TB> a, TileSplit split)
{
    using P = Phys2D<EQ>;
    using T = TB;
    constexpr int NV = P::NV, K1 = K + 1, NM = K1 * K1, L1 = 2 * K + 1;
    constexpr int FX = FilterTile<NV>::FX, FY = FilterTile<NV>::FY;
    constexpr int SX = FilterTile<NV>::SX, SY = FilterTile<NV>::SY;
    // T words per slot: with 4 variables = 4 mod 32, so the 4 cells x 4
    // variables of a 16-lane group (FP64) or the 8 x 4 of a 32-lane group
    // (FP32) hit distinct banks; with one variable odd
    constexpr int STRIDE = NV == 4 ? NM * NV + (36 - (NM * NV) % 32) % 32 : (NM | 1);
    __shared__ __align__(16) T sM[SX * SY * STRIDE];

    if (a.dt_from_ctrl && a.ctrl->done) return;
    const double dt = a.dt_from_ctrl ? a.ctrl->dt : a.dt_host;
    const double t0 = a.dt_from_ctrl ? a.ctrl->t : a.t_host;
    const double tf = t0 + (a.stage == 1 ? 0.5 : 1.0) * dt;  // time the stage output stands for

    const int tid = threadIdx.x, v = tid % NV, cidx = tid / NV;
    const int tx = cidx % FX, ty = cidx / FX;
    int64_t tbx, tby;
    if constexpr (BND) {
        ring_tile(blockIdx.x, split, tbx, tby);
    } else {
        xcd_tile(split.x1 - split.x0, gridDim.x, tbx, tby);
        tbx += split.x0;
        tby += split.y0;
    }
    const int64_t ix0 = tbx * FX, jy0 = tby * FY;
    const int64_t ix = ix0 + tx, jy = jy0 + ty;
    const bool px = a.bc[0] == BC_PERIODIC, py = a.bc[2] == BC_PERIODIC;
    const int64_t cx = slot_index(ix, a.nx, px), cy = slot_index(jy, a.ny, py);
    const bool loadable = cx >= 0 && cy >= 0;
    const bool own = ix < a.nx && jy < a.ny;
    const int oslot = (ty + 1) * SX + tx + 1;

    // own modes of variable v (registers and LDS) and the face-neighbour
    // ring's (left/right columns, bottom/top rows of the tile): both are
    // requested before either is stored, so the two trips to memory overlap
    double m0v = 0.0;
    T um[NM];
#pragma unroll
    for (int m = 0; m < NM; ++m) um[m] = (T)0;
    if (loadable) load_var2d<K, PK, TB, T>(a.us, cy * a.nx + cx, v, m0v, um);
    constexpr int NRING = 2 * FY + 2 * FX;
    const int r = tid / NV, rv = tid % NV;
    int sx = 0, sy = 0;
    if (r < FY) {
        sx = 0;
        sy = r + 1;
    } else if (r < 2 * FY) {
        sx = FX + 1;
        sy = r - FY + 1;
    } else if (r < 2 * FY + FX) {
        sx = r - 2 * FY + 1;
        sy = 0;
    } else {
        sx = r - 2 * FY - FX + 1;
        sy = FY + 1;
    }
    bool ring = false;
    T wm[NM];
#pragma unroll
    for (int m = 0; m < NM; ++m) wm[m] = (T)0;
    if (tid < NRING * NV) {
        const int64_t gx = slot_index(ix0 + sx - 1, a.nx, px), gy = slot_index(jy0 + sy - 1, a.ny, py);
        ring = gx >= 0 && gy >= 0;
        if (ring) {
            double w0;
            load_var2d<K, PK, TB, T>(a.us, gy * a.nx + gx, rv, w0, wm);
        }
    }
    if (loadable) {
#pragma unroll
        for (int m = 0; m < NM; ++m) sM[oslot * STRIDE + m * NV + v] = um[m];
    }
    if (ring) {
        const int slot = sy * SX + sx;
#pragma unroll
        for (int m = 0; m < NM; ++m) sM[slot * STRIDE + m * NV + rv] = wm[m];
    }
    __syncthreads();

    const bool lin = slot_index(ix - 1, a.nx, px) >= 0, rin = slot_index(ix + 1, a.nx, px) >= 0;
    const bool bin = slot_index(jy - 1, a.ny, py) >= 0, tin = slot_index(jy + 1, a.ny, py) >= 0;
    const double xl = a.xlo + (double)ix * a.hx, yb = a.ylo + (double)jy * a.hy;

    // cell-average state (all variables) for beta_x, beta_y and H
    T ubt[NV];
#pragma unroll
    for (int w = 0; w < NV; ++w) ubt[w] = loadable ? sM[oslot * STRIDE + w] : (T)1;
    const T bx = P::speed(ubt, 0, a.phys), by = P::speed(ubt, 1, a.phys);
    const T H = P::enthalpy(ubt, a.phys);

    T Jx[L1], Jy[L1];  // weighted sums per derivative order m = a1 + a2 (variable v)
#pragma unroll
    for (int m = 0; m < L1; ++m) Jx[m] = Jy[m] = (T)0;
    // Jumps of every mixed derivative d^a u (a1, a2 <= k) at the corners of
    // the four faces.
    if (own) {
        constexpr int AL = K1;
        // DIR 0: vertical faces (x = const), DIR 1: horizontal faces.  The
        // face side is a run-time loop index (keeps one face live at a time).
#pragma unroll
        for (int dir = 0; dir < 2; ++dir) {
#pragma unroll 1
            for (int side = 0; side < 2; ++side) {
                const bool inside = !BND || (dir == 0 ? (side ? rin : lin) : (side ? tin : bin));
                const int nslot = oslot + (dir == 0 ? (side ? 1 : -1) : (side ? SX : -SX));
                const T* UN = &sM[nslot * STRIDE + v];
                // across-face derivative values P_n^(a)(end): +1 end for
                // side 1, -1 end for side 0 (sign (-1)^(n+a)); the neighbour
                // sees the opposite end
                auto across = [&](int n, int al, int sd) -> T {
                    const double r = dtrace_r(n, al);
                    return (T)((sd || !((n + al) & 1)) ? r : -r);
                };
                // D[al][o] = sum_n (nb - own) u^{..} P_n^(al)(end), n the
                // across-face index, o the along-face index
                T D[AL][K1];
#pragma unroll
                for (int al = 0; al < AL; ++al)
#pragma unroll
                    for (int o = 0; o < K1; ++o) {
                        T go = (T)0, gn = (T)0;
#pragma unroll
                        for (int n = (al > 0 ? al : 0); n < K1; ++n) {
                            const int m = dir == 0 ? n * K1 + o : o * K1 + n;
                            if (!mode_kept<K, PK>(m)) continue;
                            go += um[m] * across(n, al, side);
                            if (inside) gn += UN[m * NV] * across(n, al, 1 - side);
                        }
                        D[al][o] = inside ? gn - go : go;
                    }
                // outside the domain: the ghost at the two corners of this face
                int gk[2] = {0, 0};
                bool grf[2] = {false, false};
                T gst[2] = {(T)0, (T)0};
                if (!inside) {
                    const int fside = 2 * dir + side;
#pragma unroll
                    for (int cc = 0; cc < 2; ++cc) {
                        const double xc = dir == 0 ? xl + (side ? a.hx : 0.0) : xl + (cc ? a.hx : 0.0);
                        const double yc = dir == 0 ? yb + (cc ? a.hy : 0.0) : yb + (side ? a.hy : 0.0);
                        bool rf;
                        gk[cc] = boundary_kind(a, fside, xc, yc, tf, &rf);
                        grf[cc] = rf;
                        gst[cc] = gk[cc] ? (T)boundary_state(a, fside, gk[cc], v) : (T)0;
                    }
                }
#pragma unroll
                for (int cc = 0; cc < 2; ++cc)
#pragma unroll
                    for (int al = 0; al < AL; ++al)
#pragma unroll
                        for (int bl = 0; bl < AL; ++bl) {
                            // al: across-face derivative order, bl: along-face
                            T sum = (T)0;
#pragma unroll
                            for (int o = (bl > 0 ? bl : 0); o < K1; ++o)
                                sum += D[al][o] * (T)dtr(o, bl, cc);
                            T j = fabs(sum);
                            if (!inside) {
                                if (gk[cc])
                                    j = (al == 0 && bl == 0) ? fabs(gst[cc] - sum) : fabs(sum);
                                else if (grf[cc])
                                    j = (((al & 1) != 0) != (v == 1 + dir)) ? (T)2 * fabs(sum) : (T)0;
                                else
                                    j = (T)0;
                            }
                            const int a1 = dir == 0 ? al : bl, a2 = dir == 0 ? bl : al;
                            if (dir == 0)
                                Jx[a1 + a2] += (T)(0.5 * a.jsx[a1 * 4 + a2]) * j;
                            else
                                Jy[a1 + a2] += (T)(0.5 * a.jsy[a1 * 4 + a2]) * j;
                        }
            }
        }
    }
    // running partial sums over the derivative order, then the maximum over
    // the variables (in variable order, as a sequential loop would take it)
    T best[L1];
    {
        T sx = (T)0, sy = (T)0;
        const int base = tid - v;
#pragma unroll
        for (int l = 0; l < L1; ++l) {
            sx += Jx[l];
            sy += Jy[l];
            const T sv = (T)a.cfmx * bx * sx + (T)a.cfmy * by * sy;
            T bl = sv;
#pragma unroll
            for (int w = 0; w < NV; ++w) {
                const T o = NV > 1 ? __shfl(sv, base + w, 64) : sv;
                bl = (w == 0 || o > bl) ? o : bl;
            }
            best[l] = bl;
        }
    }
    if (!own) return;
    const int64_t cell = jy * a.nx + ix;
    const T coef = (T)dt * (T)(a.inv_hx * a.inv_hy) * trcp<T>(H);
    T E[L1];
    E[0] = (T)0;
#pragma unroll
    for (int l = 1; l < L1; ++l) E[l] = coef * best[l];
    if (a.E_out && v == 0) {
#pragma unroll
        for (int l = 0; l < L1; ++l) a.E_out[cell * L1 + l] = (double)E[l];
    }
    T f[L1];
#pragma unroll
    for (int l = 1; l < L1; ++l) f[l] = texp<T>(-E[l]);
    a.out.m0[v * a.out.s0 + cell] = m0v;
    double sabs = 0.0;
#pragma unroll
    for (int p = 0; p < K1; ++p)
#pragma unroll
        for (int q = 0; q < K1; ++q) {
            if ((p == 0 && q == 0) || (PK && p + q > K)) continue;
            const int m = p * K1 + q;
            const T val = um[m] * f[p + q];
            sabs += fabs((double)val);
            a.out.hi[v * a.out.sv + (mode_plane<K, PK>(m) - 1) * a.out.sl + cell] = val;
        }
    // positivity limiter: list the cells its screen does not clear
    if constexpr (EQ == EULER) {
        if (a.pp && !pp2_clear_lanes<TB>(m0v, sabs, tid - v, a.phys.gamma) && v == 0) {
            const unsigned long long slot = atomicAdd(a.pcount, 1ull);
            if ((long long)slot < a.pcap) a.pcell[slot] = cell;
        }
    }
}

// Hybrid limiter, pass B2, over the troubled list: u^{pq} <- [w + (1 - w) exp(-E^{p+q})] u^{pq},
// then (Euler, pp.on) the positivity limiter's screen on the blended cell:
// the cells it does not clear are appended to the limiter's list (pcell),
// which pp2d_kernel limits next.  One wavefront per troubled cell: lane
// l < NV (K+1)^2 holds coefficient (variable l / (K+1)^2, mode l % (K+1)^2).
template <int K, int NV, typename TB, bool PK>
__global__ __launch_bounds__(256) void blend2d_kernel(StateView<TB> out, const unsigned int* count,
                                                      const long long* tcell, const double* tdata,
                                                      const unsigned long long* eta_bits,
                                                      const Ctrl* ctrl, int from_ctrl, long long cap,
                                                      PPArgs pp, unsigned long long* pcount,
                                                      long long* pcell, long long pcap)
{
    constexpr int K1 = K + 1, NM = K1 * K1, L1 = 2 * K + 1, NC = NV * NM;
    __shared__ double sc[4][NV == 4 ? NC : 1];
    if (from_ctrl && ctrl->done) return;
    unsigned int cnt = *count;
    if ((long long)cnt > cap) cnt = (unsigned int)cap;
    const double M = __longlong_as_double((long long)*eta_bits);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int v = lane / NM, m = lane % NM, p = m / K1, q = m % K1;
    const bool mine = lane < NC && m > 0 && mode_kept<K, PK>(m);
    const int64_t off = mine ? v * out.sv + (mode_plane<K, PK>(m) - 1) * out.sl : 0;
    for (unsigned int i = blockIdx.x * 4 + wv; i < cnt; i += gridDim.x * 4) {
        const long long c = tcell[i];
        const double* rec = tdata + (size_t)i * L1;
        const double w = (M - rec[0]) / (M - 1.0);
        double cf = 0.0;
        if (mine) {
            const TB f = (TB)(w + (1.0 - w) * exp(-rec[p + q]));
            cf = (double)(out.hi[off + c] * f);
            out.hi[off + c] = (TB)cf;
        } else if (lane < NC && m == 0) {
            cf = out.m0[v * out.s0 + c];
        }
        if constexpr (NV == 4) {
            if (pp.on) {
                // the screen pp2_wave starts with, on the blended cell
                double* cw = sc[wv];
                if (lane < NC) cw[lane] = cf;
                wave_lds_sync();
                double ub[4], sabs[4];
#pragma unroll
                for (int vv = 0; vv < 4; ++vv) {
                    ub[vv] = cw[vv * NM];
                    double t = 0.0;
#pragma unroll
                    for (int mm = 1; mm < NM; ++mm) t += fabs(cw[vv * NM + mm]);
                    sabs[vv] = t;
                }
                if (!pp2_clear<TB>(ub, sabs, pp.phys.gamma) && lane == 0) {
                    const unsigned long long slot = atomicAdd(pcount, 1ull);
                    if ((long long)slot < pcap) pcell[slot] = c;
                }
                wave_lds_sync();  // the next cell rewrites the block
            }
        }
    }
}

// Positivity limiter over the cells the post-stage kernels listed (or over
// every cell when count is null), in place; one wavefront per cell.
template <int K, typename TB, bool PK>
__global__ __launch_bounds__(256) void pp2d_kernel(StateView<TB> u, long long ncell,
                                                   const unsigned long long* count, const long long* cells,
                                                   long long cap, const Ctrl* ctrl, int from_ctrl, PPArgs pp)
{
    constexpr int K1 = K + 1, NM = K1 * K1, NC = 4 * NM;
    __shared__ double sc[4][NC];
    if (from_ctrl && ctrl->done) return;
    long long cnt = ncell;
    if (count) {
        const unsigned long long c = *count;
        cnt = (long long)c < cap ? (long long)c : cap;
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int v = lane / NM, m = lane % NM;
    const bool mine = lane < NC && m > 0 && mode_kept<K, PK>(m);
    const int64_t off = mine ? v * u.sv + (mode_plane<K, PK>(m) - 1) * u.sl : 0;
    for (long long i = (long long)blockIdx.x * 4 + wv; i < cnt; i += (long long)gridDim.x * 4) {
        const long long c = count ? cells[i] : i;
        double cf = 0.0;
        if (mine)
            cf = (double)u.hi[off + c];
        else if (lane < NC && m == 0)
            cf = u.m0[v * u.s0 + c];
        if (pp2_wave<K, PK, TB>(sc[wv], cf, lane, pp.phys.gamma, pp.reject) && mine)
            u.hi[off + c] = (TB)cf;
    }
}

// -------------------------------------------------------------------------
// Hybrid limiter, pass A (Algorithm 1): the jump indicator
//   eta = max_v (Jx0_v / (2 hx) + Jy0_v / (2 hy)),
// Jx0, Jy0 the trapezoid edge averages of the value jumps over the vertical
// and horizontal faces, for every cell of a.us (read only); the domain
// maximum of eta (a.eta_acc), the troubled cells (eta > 1: a.tcell, with eta
// in the first entry of each a.tdata record), and, with the positivity
// limiter, the cells that stay unfiltered and whose screen fails (a.pcell).
// The exponents of the troubled cells are computed by troubled2d_kernel.
// Mapping as filter2d: one lane per (cell, variable), FX x FY cells per
// workgroup (FX x 2 FY, two cells per lane, when it reads the corner values
// the stage kernel handed over); each lane evaluates its variable at the
// four corners of its cell (the values P_p(+-1) P_q(+-1) = +-1, summed in the
// order p, q), the tile's ring cells their two facing corners, and the
// corner values meet in LDS.
// -------------------------------------------------------------------------
// Rows of cells per lane of the indicator: two when it reads the corner
// values (the time steps), so each lane has twice the loads in flight and a
// workgroup's tile is FX x 2 FY cells; one when it forms them from the state.
template <bool CORNER>
struct IndicatorRows {
    static constexpr int RPL = CORNER ? 2 : 1;
};

template <int EQ, int K, typename TB, bool PK, bool CORNER>
__global__ __launch_bounds__(256) void indicator2d_kernel(Args2D<TB> a)
{
    using P = Phys2D<EQ>;
    using T = TB;
    constexpr int NV = P::NV, K1 = K + 1, NM = K1 * K1, L1 = 2 * K + 1;
    constexpr int RPL = IndicatorRows<CORNER>::RPL;
    constexpr int FX = FilterTile<NV>::FX, FY = FilterTile<NV>::FY, TY = RPL * FY;
    constexpr int NRING = 2 * TY + 2 * FX;
    static_assert(NRING * NV <= 256, "one lane per (ring cell, variable)");
    // corner values: own cells [corner sx + 2 sy][cell][var]; ring cells
    // [the two facing corners][ring index][var] (consecutive lanes,
    // consecutive words)
    constexpr int CS = FX * TY * NV, RS = NRING * NV;
    __shared__ T sC[4 * CS];
    __shared__ T sR[2 * RS];

    if (a.dt_from_ctrl && a.ctrl->done) return;
    const double dt = a.dt_from_ctrl ? a.ctrl->dt : a.dt_host;
    const double t0 = a.dt_from_ctrl ? a.ctrl->t : a.t_host;
    const double tf = t0 + (a.stage == 1 ? 0.5 : 1.0) * dt;  // time the stage output stands for

    // lane (cell, variable) of the first row band; the lane also takes the
    // cell FY rows above for RPL = 2
    const int tid = threadIdx.x, v = tid % NV, cidx = tid / NV;
    const int tx = cidx % FX, ty0 = cidx / FX;
    int64_t tbx, tby;
    xcd_tile((a.nx + FX - 1) / FX, gridDim.x, tbx, tby);
    const int64_t ix0 = tbx * FX, jy0 = tby * TY;
    const int64_t ix = ix0 + tx;
    const bool px = a.bc[0] == BC_PERIODIC, py = a.bc[2] == BC_PERIODIC;
    // a slot past the mesh in a ragged tile holds the periodic image (the
    // face neighbour of the last own cell), or nothing
    const int64_t cx = slot_index(ix, a.nx, px);
    int64_t jy[RPL];
    bool own[RPL];
    double m0v[RPL];
    T um[RPL][NM];
    {
        T cv[RPL][4];
        bool loadable[RPL];
#pragma unroll
        for (int h = 0; h < RPL; ++h) {
            jy[h] = jy0 + ty0 + h * FY;
            own[h] = ix < a.nx && jy[h] < a.ny;
            const int64_t cy = slot_index(jy[h], a.ny, py);
            loadable[h] = cx >= 0 && cy >= 0;
            m0v[h] = 0.0;
#pragma unroll
            for (int m = 0; m < NM; ++m) um[h][m] = (T)0;
            if (loadable[h]) {
                const int64_t c0 = cy * a.nx + cx;
                if constexpr (CORNER) {
#pragma unroll
                    for (int c = 0; c < 4; ++c) cv[h][c] = a.corner[(c * NV + v) * a.cstride + c0];
                } else {
                    load_var2d<K, PK, TB, T>(a.us, c0, v, m0v[h], um[h]);
#pragma unroll
                    for (int c = 0; c < 4; ++c) cv[h][c] = corner2d<K, PK, T>(um[h], c & 1, c >> 1);
                }
            }
        }
        // (the loads of all rows are requested before any is stored)
#pragma unroll
        for (int h = 0; h < RPL; ++h)
            if (loadable[h]) {
                const int cl = (ty0 + h * FY) * FX + tx;
#pragma unroll
                for (int c = 0; c < 4; ++c) sC[c * CS + cl * NV + v] = cv[h][c];
            }
    }
    if (tid < NRING * NV) {
        const int r = tid / NV, rv = tid % NV;
        int g, i;  // 0 left column, 1 right column, 2 bottom row, 3 top row
        if (r < TY) { g = 0; i = r; }
        else if (r < 2 * TY) { g = 1; i = r - TY; }
        else if (r < 2 * TY + FX) { g = 2; i = r - 2 * TY; }
        else { g = 3; i = r - 2 * TY - FX; }
        const int64_t gx = g == 0 ? ix0 - 1 : g == 1 ? ix0 + FX : ix0 + i;
        const int64_t gy = g == 2 ? jy0 - 1 : g == 3 ? jy0 + TY : jy0 + i;
        const int64_t hx_ = slot_index(gx, a.nx, px), hy_ = slot_index(gy, a.ny, py);
        if (hx_ >= 0 && hy_ >= 0) {
            const int64_t c1 = hy_ * a.nx + hx_;
            // facing corners, ordered along the face: the left column's
            // right corners (bottom, top), the right column's left corners,
            // the bottom row's top corners (left, right), the top row's
            // bottom corners
            if constexpr (CORNER) {
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const int sx = g == 0 ? 1 : g == 1 ? 0 : c, sy = g == 2 ? 1 : g == 3 ? 0 : c;
                    sR[c * RS + r * NV + rv] = a.corner[((sx + 2 * sy) * NV + rv) * a.cstride + c1];
                }
            } else {
                double w0;
                T wm[NM];
                load_var2d<K, PK, TB, T>(a.us, c1, rv, w0, wm);
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const int sx = g == 0 ? 1 : g == 1 ? 0 : c, sy = g == 2 ? 1 : g == 3 ? 0 : c;
                    sR[c * RS + r * NV + rv] = corner2d<K, PK, T>(wm, sx, sy);
                }
            }
        }
    }
    __syncthreads();

    T eta[RPL];
    double zmax = 0.0;
#pragma unroll
    for (int h = 0; h < RPL; ++h) {
        const int ty = ty0 + h * FY;
        eta[h] = (T)0;
        if (own[h]) {
            const bool lin = slot_index(ix - 1, a.nx, px) >= 0, rin = slot_index(ix + 1, a.nx, px) >= 0;
            const bool bin = slot_index(jy[h] - 1, a.ny, py) >= 0, tin = slot_index(jy[h] + 1, a.ny, py) >= 0;
            const double xl = a.xlo + (double)ix * a.hx, yb = a.ylo + (double)jy[h] * a.hy;
            // the neighbour's value at corner c of the face (dir, side): from
            // the tile or its ring
            auto nb_corner = [&](int dir, int side, int c) -> T {
                if (dir == 0) {
                    const int nx_ = tx + (side ? 1 : -1);
                    if (nx_ >= 0 && nx_ < FX) return sC[((side ? 0 : 1) + 2 * c) * CS + (ty * FX + nx_) * NV + v];
                    const int r = side ? TY + ty : ty;
                    return sR[c * RS + r * NV + v];
                }
                const int ny_ = ty + (side ? 1 : -1);
                if (ny_ >= 0 && ny_ < TY) return sC[(c + (side ? 0 : 2)) * CS + (ny_ * FX + tx) * NV + v];
                const int r = side ? 2 * TY + FX + tx : 2 * TY + tx;
                return sR[c * RS + r * NV + v];
            };
            T jx = (T)0, jyv = (T)0;
#pragma unroll
            for (int side = 0; side < 2; ++side)
#pragma unroll
                for (int dir = 0; dir < 2; ++dir) {
                    const bool inside = dir == 0 ? (side ? rin : lin) : (side ? tin : bin);
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        // own corner of this face
                        const int sx = dir == 0 ? side : c, sy = dir == 0 ? c : side;
                        const T in = sC[(sx + 2 * sy) * CS + (ty * FX + tx) * NV + v];
                        T j;
                        if (inside) {
                            j = fabs(nb_corner(dir, side, c) - in);
                        } else {
                            const double xc = xl + (sx ? a.hx : 0.0), yc = yb + (sy ? a.hy : 0.0);
                            bool rf;
                            const int kind = boundary_kind(a, 2 * dir + side, xc, yc, tf, &rf);
                            if (kind)
                                j = fabs((T)boundary_state(a, 2 * dir + side, kind, v) - in);
                            else if (rf)
                                j = (v == 1 + dir) ? (T)2 * fabs(in) : (T)0;
                            else
                                j = (T)0;
                        }
                        if (dir == 0)
                            jx += (T)0.5 * j;
                        else
                            jyv += (T)0.5 * j;
                    }
                }
            eta[h] = jx * (T)(0.5 * a.inv_hx) + jyv * (T)(0.5 * a.inv_hy);
        }
        {
            const int base = tid - v;
            T e = eta[h];
#pragma unroll
            for (int w = 0; w < NV; ++w) {
                const T o = NV > 1 ? __shfl(eta[h], base + w, 64) : eta[h];
                e = (w == 0 || o > e) ? o : e;
            }
            eta[h] = e;
        }
        const double z = own[h] ? (double)eta[h] : 0.0;
        zmax = (z > zmax || z != z) ? z : zmax;
    }
    // max eta over the grid: every lane reaches the wave reduction
    const double z = wave_max(zmax);
    if ((tid & 63) == 0) atomic_max_nonneg(a.eta_acc, z);
#pragma unroll
    for (int h = 0; h < RPL; ++h) {
        if (!own[h]) continue;
        const int64_t cell = jy[h] * a.nx + ix;
        if (a.E_out && v == 0) {
#pragma unroll
            for (int l = 0; l < L1; ++l) a.E_out[cell * L1 + l] = 0.0;
        }
        if constexpr (EQ == EULER) {
            // positivity limiter: cells that stay unfiltered (eta <= 1) are
            // final now; troubled cells are screened after their blend
            if (a.pp) {
                bool fail;
                if constexpr (CORNER) {
                    fail = a.ppfail[cell] != 0;  // the stage kernel's screen
                } else {
                    double sabs = 0.0;
#pragma unroll
                    for (int m = 1; m < NM; ++m) sabs += fabs((double)um[h][m]);
                    fail = !pp2_clear_lanes<TB>(m0v[h], sabs, tid - v, a.phys.gamma);
                }
                if (!(eta[h] > (T)1) && fail && v == 0) {
                    const unsigned long long slot = atomicAdd(a.pcount, 1ull);
                    if ((long long)slot < a.pcap) a.pcell[slot] = cell;
                }
            }
        }
        if (v == 0) {
            if (a.eta_out) a.eta_out[cell] = (double)eta[h];
            if (eta[h] > (T)1) {
                const unsigned int slot = atomicAdd(a.tcount, 1u);
                if ((long long)slot < a.tcap) {
                    a.tcell[slot] = cell;
                    a.tdata[(size_t)slot * L1] = (double)eta[h];
                }
            }
        }
    }
}

// -------------------------------------------------------------------------
// Hybrid limiter, pass B1: for each troubled cell of the list (one wavefront
// per cell) the damping exponents of the jump filter, from the jumps of every
// mixed derivative d^a u (a1, a2 <= k) at the corners of the four faces
// (para:damp22d)-(para:damp22d1) with the systems rule (maximum over the
// variables), into the cell's a.tdata record (E^1..E^{2k} after eta).  The
// state is only read: every troubled cell's exponents come from the
// unfiltered stage output (Jacobi), and blend2d_kernel applies them after.
// Lanes: l = v (k+1)^2 + al (k+1) + bl takes the derivative orders (al across
// a face, bl along it) of variable v on every face; l = v (k+1)^2 + m loads
// coefficient m of variable v.
// -------------------------------------------------------------------------
template <int EQ, int K, typename TB, bool PK>
__global__ __launch_bounds__(256) void troubled2d_kernel(Args2D<TB> a)
{
    using P = Phys2D<EQ>;
    using T = TB;
    constexpr int NV = P::NV, K1 = K + 1, NM = K1 * K1, L1 = 2 * K + 1, NC = NV * NM;
    static_assert(NC <= 64, "one lane per coefficient");
    // per wavefront: the modes of the cell and of its four face neighbours
    // (own, left, right, bottom, top), the per-lane weighted jump sums and the
    // per-variable sums
    struct WaveLds {
        T u[5][NC];
        T wx[NC], wy[NC];
        T sv[NV][L1];
    };
    __shared__ WaveLds sh[4];
    if (a.dt_from_ctrl && a.ctrl->done) return;
    const double dt = a.dt_from_ctrl ? a.ctrl->dt : a.dt_host;
    const double t0 = a.dt_from_ctrl ? a.ctrl->t : a.t_host;
    const double tf = t0 + (a.stage == 1 ? 0.5 : 1.0) * dt;
    unsigned int cnt = *a.tcount;
    if ((long long)cnt > a.tcap) cnt = (unsigned int)a.tcap;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    WaveLds& L = sh[wv];
    const int v = lane / NM, m = lane % NM;
    const int al = m / K1, bl = m % K1;  // derivative orders of this lane
    const bool act = lane < NC;
    const bool px = a.bc[0] == BC_PERIODIC, py = a.bc[2] == BC_PERIODIC;
    for (unsigned int i = blockIdx.x * 4 + wv; i < cnt; i += gridDim.x * 4) {
        const long long c = a.tcell[i];
        const int64_t ix = c % a.nx, jy = c / a.nx;
        const int64_t nbx[4] = {slot_index(ix - 1, a.nx, px), slot_index(ix + 1, a.nx, px), ix, ix};
        const int64_t nby[4] = {jy, jy, slot_index(jy - 1, a.ny, py), slot_index(jy + 1, a.ny, py)};
        // loads: coefficient m of variable v of the cell and its neighbours
        if (act) {
            const bool kept = mode_kept<K, PK>(m);
            const int64_t off = m == 0 ? v * a.us.s0 : v * a.us.sv + (mode_plane<K, PK>(m > 0 ? m : 1) - 1) * a.us.sl;
            for (int nb = 0; nb < 5; ++nb) {
                const int64_t gx = nb == 0 ? ix : nbx[nb - 1], gy = nb == 0 ? jy : nby[nb - 1];
                T val = (T)0;
                if (gx >= 0 && gy >= 0 && kept) {
                    const int64_t cc = gy * a.nx + gx;
                    val = m == 0 ? (T)a.us.m0[off + cc] : (T)a.us.hi[off + cc];
                }
                L.u[nb][lane] = val;
            }
        }
        wave_lds_sync();
        // jumps of d^(al, bl) (x faces) and d^(bl, al) (y faces) of variable v
        T wxs = (T)0, wys = (T)0;
        if (act) {
            const double xl = a.xlo + (double)ix * a.hx, yb = a.ylo + (double)jy * a.hy;
            const T* U = &L.u[0][v * NM];
#pragma unroll
            for (int dir = 0; dir < 2; ++dir)
#pragma unroll
                for (int side = 0; side < 2; ++side) {
                    const int nb = 1 + 2 * dir + side;
                    const bool inside = (dir == 0 ? nbx[2 * dir + side] : nby[2 * dir + side]) >= 0;
                    const T* UN = &L.u[nb][v * NM];
                    auto across = [&](int n, int sd) -> T {
                        const double r = dtrace_r(n, al);
                        return (T)((sd || !((n + al) & 1)) ? r : -r);
                    };
                    T D[K1];
#pragma unroll
                    for (int o = 0; o < K1; ++o) {
                        T go = (T)0, gn = (T)0;
#pragma unroll
                        for (int n = 0; n < K1; ++n) {
                            if (n < al) continue;
                            const int mm = dir == 0 ? n * K1 + o : o * K1 + n;
                            go += U[mm] * across(n, side);
                            if (inside) gn += UN[mm] * across(n, 1 - side);
                        }
                        D[o] = inside ? gn - go : go;
                    }
#pragma unroll
                    for (int cc = 0; cc < 2; ++cc) {
                        T sum = (T)0;
#pragma unroll
                        for (int o = 0; o < K1; ++o)
                            if (o >= bl) sum += D[o] * (T)dtr(o, bl, cc);
                        T j = fabs(sum);
                        if (!inside) {
                            const double xc = dir == 0 ? xl + (side ? a.hx : 0.0) : xl + (cc ? a.hx : 0.0);
                            const double yc = dir == 0 ? yb + (cc ? a.hy : 0.0) : yb + (side ? a.hy : 0.0);
                            bool rf;
                            const int kind = boundary_kind(a, 2 * dir + side, xc, yc, tf, &rf);
                            if (kind)
                                j = (al == 0 && bl == 0) ? fabs((T)boundary_state(a, 2 * dir + side, kind, v) - sum)
                                                         : fabs(sum);
                            else if (rf)
                                j = (((al & 1) != 0) != (v == 1 + dir)) ? (T)2 * fabs(sum) : (T)0;
                            else
                                j = (T)0;
                        }
                        if (dir == 0)
                            wxs += (T)(0.5 * a.jsx[al * 4 + bl]) * j;
                        else
                            wys += (T)(0.5 * a.jsy[bl * 4 + al]) * j;
                    }
                }
            L.wx[lane] = wxs;
            L.wy[lane] = wys;
        }
        wave_lds_sync();
        // per variable: running sums over the derivative order l = al + bl,
        // weighted by the coefficient's mesh factors and wave speeds
        if (lane < NV) {
            T ub[NV];
#pragma unroll
            for (int w = 0; w < NV; ++w) ub[w] = L.u[0][w * NM];
            const T bx = P::speed(ub, 0, a.phys), by = P::speed(ub, 1, a.phys);
            T sx = (T)0, sy = (T)0;
#pragma unroll
            for (int l = 0; l < L1; ++l) {
#pragma unroll
                for (int x = 0; x < K1; ++x) {
                    const int y = l - x;
                    if (y < 0 || y >= K1) continue;
                    sx += L.wx[lane * NM + x * K1 + y];
                    sy += L.wy[lane * NM + x * K1 + y];
                }
                L.sv[lane][l] = (T)a.cfmx * bx * sx + (T)a.cfmy * by * sy;
            }
        }
        wave_lds_sync();
        T ubt[NV];
#pragma unroll
        for (int w = 0; w < NV; ++w) ubt[w] = L.u[0][w * NM];
        const T H = P::enthalpy(ubt, a.phys);
        const T coef = (T)dt * (T)(a.inv_hx * a.inv_hy) * trcp<T>(H);
        // E^l = coef max_v sv[v][l], l = 1..2k, after eta in the record
        if (lane < L1) {
            T bl_ = L.sv[0][lane];
#pragma unroll
            for (int vv = 1; vv < NV; ++vv) bl_ = L.sv[vv][lane] > bl_ ? L.sv[vv][lane] : bl_;
            const double E = lane == 0 ? 0.0 : (double)(coef * bl_);
            if (lane > 0) a.tdata[(size_t)i * L1 + lane] = E;
            if (a.E_out) a.E_out[c * L1 + lane] = E;
        }
        wave_lds_sync();  // the next cell rewrites the block
    }
}

// P^k exchange conversion: the FP64 exchange layout [var][p (k+1) + q][cell]
// (every Q^k mode) <-> the compact internal P^k planes.  To the device the
// modes p + q > k are dropped (the L2 projection onto P^k, the Legendre
// basis being orthogonal); from the device they are written as zeros.
template <typename TB>
__global__ __launch_bounds__(256) void convert_pk2d_kernel(int to_internal, int k, int64_t ncell,
                                                           int64_t total, const double* ext_in,
                                                           double* ext_out, StateView<TB> v)
{
    const int K1 = k + 1, NM = K1 * K1;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = i % ncell;
        const int64_t rest = i / ncell;
        const int m = (int)(rest % NM);
        const int var = (int)(rest / NM);
        const int p = m / K1, q = m % K1;
        if (p + q > k) {
            if (!to_internal) ext_out[i] = 0.0;
            continue;
        }
        const int plane = p * K1 - p * (p - 1) / 2 + q;
        if (plane == 0) {
            double* d = v.m0 + var * v.s0 + c;
            if (to_internal)
                *d = ext_in[i];
            else
                ext_out[i] = *d;
        } else {
            TB* d = v.hi + var * v.sv + (int64_t)(plane - 1) * v.sl + c;
            if (to_internal)
                *d = (TB)ext_in[i];
            else
                ext_out[i] = (double)*d;
        }
    }
}

template <typename TB>
hipError_t launch_convert_pk2d(int to_internal, int nv, int k, int64_t ncell, const double* ext,
                               StateView<TB> v, hipStream_t st)
{
    const int64_t total = (int64_t)nv * (k + 1) * (k + 1) * ncell;
    int64_t g = (total + 255) / 256;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    hipLaunchKernelGGL((convert_pk2d_kernel<TB>), dim3((unsigned)g), dim3(256), 0, st, to_internal, k,
                       ncell, total, ext, const_cast<double*>(ext), v);
    return hipGetLastError();
}

template <int EQ, typename TB>
__global__ __launch_bounds__(256) void maxwave2d_kernel(StateView<TB> u, int64_t ncell, double ihx,
                                                        double ihy, PhysParams phys,
                                                        unsigned long long* acc, Ctrl* err)
{
    constexpr int NV = Phys2D<EQ>::NV;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double lam = 0.0;
    if (c < ncell) {
        double ub[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) ub[v] = u.m0[v * u.s0 + c];
        lam = Phys2D<EQ>::cfl(ub, ihx, ihy, phys);
        if (EQ == EULER) {
            const double p = Phys2D<EULER>::pressure(ub, phys);
            if (!(ub[0] > 0.0) || !(p > 0.0)) latch_error(err, (isfinite(ub[0]) && isfinite(p)) ? -5 : -4, c);
        }
        if (!isfinite(lam)) latch_error(err, -4, c);
    }
    lam = wave_max(lam);
    if ((threadIdx.x & 63) == 0) atomic_max_nonneg(acc, lam);
}

// ------------------------------------------------------------ launchers --
template <typename TB>
hipError_t launch_stage2d(int eq, int k, const Args2D<TB>& a, hipStream_t st)
{
    const int fx = eq == ADV ? StageTile<1>::FX : StageTile<4>::FX;
    const int fy = eq == ADV ? StageTile<1>::FY : StageTile<4>::FY;
    dim3 grid((unsigned)(((a.nx + fx - 1) / fx) * ((a.ny + fy - 1) / fy))), block(256);
#define DG_CASE(E_, K_)                                                                   \
    if (eq == E_ && k == K_) {                                                            \
        const bool hx = E_ == EULER && a.phys.flux != 0;                                  \
        if (a.pk && hx)                                                                   \
            hipLaunchKernelGGL((stage2d_kernel<E_, K_, TB, (K_ > 0), (E_ == EULER)>), grid, block, 0, st, a); \
        else if (a.pk)                                                                    \
            hipLaunchKernelGGL((stage2d_kernel<E_, K_, TB, (K_ > 0), false>), grid, block, 0, st, a); \
        else if (hx)                                                                      \
            hipLaunchKernelGGL((stage2d_kernel<E_, K_, TB, false, (E_ == EULER)>), grid, block, 0, st, a); \
        else                                                                              \
            hipLaunchKernelGGL((stage2d_kernel<E_, K_, TB, false, false>), grid, block, 0, st, a); \
        return hipGetLastError();                                                         \
    }
    DG_CASE(ADV, 0) DG_CASE(ADV, 1) DG_CASE(ADV, 2) DG_CASE(ADV, 3)
    DG_CASE(EULER, 0) DG_CASE(EULER, 1) DG_CASE(EULER, 2) DG_CASE(EULER, 3)
#undef DG_CASE
    return hipErrorInvalidValue;
}

template <typename TB>
hipError_t launch_filter2d(int eq, int k, const Args2D<TB>& a, hipStream_t st)
{
    const int fx = eq == ADV ? FilterTile<1>::FX : FilterTile<4>::FX;
    const int fy = eq == ADV ? FilterTile<1>::FY : FilterTile<4>::FY;
    TileSplit t;
    t.gx = (a.nx + fx - 1) / fx;
    t.gy = (a.ny + fy - 1) / fy;
    const bool px = a.bc[0] == BC_PERIODIC, py = a.bc[2] == BC_PERIODIC;
    t.x0 = px ? 0 : (t.gx < 1 ? t.gx : 1);
    t.x1 = px ? t.gx : (t.gx - 1 > t.x0 ? t.gx - 1 : t.x0);
    t.y0 = py ? 0 : (t.gy < 1 ? t.gy : 1);
    t.y1 = py ? t.gy : (t.gy - 1 > t.y0 ? t.gy - 1 : t.y0);
    const dim3 gi((unsigned)t.interior()), gb((unsigned)t.boundary()), block(256);
    // interior tiles, then the boundary tiles (disjoint cells, same stream)
#define DG_LAUNCH(E_, K_, PK_)                                                                     \
    do {                                                                                           \
        if (gi.x) hipLaunchKernelGGL((filter2d_kernel<E_, K_, TB, PK_, false>), gi, block, 0, st, a, t); \
        if (gb.x) hipLaunchKernelGGL((filter2d_kernel<E_, K_, TB, PK_, true>), gb, block, 0, st, a, t);  \
    } while (0)
#define DG_CASE(E_, K_)                                                                            \
    if (eq == E_ && k == K_) {                                                                     \
        if (a.pk)                                                                                  \
            DG_LAUNCH(E_, K_, (K_ > 0));                                                           \
        else                                                                                       \
            DG_LAUNCH(E_, K_, false);                                                              \
        return hipGetLastError();                                                                  \
    }
    DG_CASE(ADV, 0) DG_CASE(ADV, 1) DG_CASE(ADV, 2) DG_CASE(ADV, 3)
    DG_CASE(EULER, 0) DG_CASE(EULER, 1) DG_CASE(EULER, 2) DG_CASE(EULER, 3)
#undef DG_CASE
#undef DG_LAUNCH
    return hipErrorInvalidValue;
}

template <typename TB>
hipError_t launch_indicator2d(int eq, int k, const Args2D<TB>& a, hipStream_t st)
{
    const int fx = eq == ADV ? FilterTile<1>::FX : FilterTile<4>::FX;
    const int fy = (eq == ADV ? FilterTile<1>::FY : FilterTile<4>::FY) *
                   (a.corner ? IndicatorRows<true>::RPL : IndicatorRows<false>::RPL);
    dim3 grid((unsigned)(((a.nx + fx - 1) / fx) * ((a.ny + fy - 1) / fy))), block(256);
    // corner values handed over by the stage kernel (dg_run), or the state
#define DG_CASE(E_, K_)                                                                            \
    if (eq == E_ && k == K_) {                                                                     \
        if (a.pk && a.corner)                                                                      \
            hipLaunchKernelGGL((indicator2d_kernel<E_, K_, TB, (K_ > 0), true>), grid, block, 0, st, a); \
        else if (a.pk)                                                                             \
            hipLaunchKernelGGL((indicator2d_kernel<E_, K_, TB, (K_ > 0), false>), grid, block, 0, st, a); \
        else if (a.corner)                                                                         \
            hipLaunchKernelGGL((indicator2d_kernel<E_, K_, TB, false, true>), grid, block, 0, st, a); \
        else                                                                                       \
            hipLaunchKernelGGL((indicator2d_kernel<E_, K_, TB, false, false>), grid, block, 0, st, a); \
        return hipGetLastError();                                                                  \
    }
    DG_CASE(ADV, 0) DG_CASE(ADV, 1) DG_CASE(ADV, 2) DG_CASE(ADV, 3)
    DG_CASE(EULER, 0) DG_CASE(EULER, 1) DG_CASE(EULER, 2) DG_CASE(EULER, 3)
#undef DG_CASE
    return hipErrorInvalidValue;
}

template <typename TB>
hipError_t launch_troubled2d(int eq, int k, const Args2D<TB>& a, hipStream_t st)
{
    // one wavefront per troubled cell, 4 per workgroup, grid-stride beyond
    // 4096 workgroups (the list's length is only known on the device)
    int64_t g = (a.tcap + 3) / 4;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
#define DG_CASE(E_, K_)                                                                            \
    if (eq == E_ && k == K_) {                                                                     \
        if (a.pk)                                                                                  \
            hipLaunchKernelGGL((troubled2d_kernel<E_, K_, TB, (K_ > 0)>), dim3((unsigned)g), dim3(256), 0, st, a); \
        else                                                                                       \
            hipLaunchKernelGGL((troubled2d_kernel<E_, K_, TB, false>), dim3((unsigned)g), dim3(256), 0, st, a);    \
        return hipGetLastError();                                                                  \
    }
    DG_CASE(ADV, 0) DG_CASE(ADV, 1) DG_CASE(ADV, 2) DG_CASE(ADV, 3)
    DG_CASE(EULER, 0) DG_CASE(EULER, 1) DG_CASE(EULER, 2) DG_CASE(EULER, 3)
#undef DG_CASE
    return hipErrorInvalidValue;
}

template <typename TB>
hipError_t launch_blend2d(int nv, int k, const Args2D<TB>& a, PPArgs pp, hipStream_t st)
{
    // one wavefront per troubled cell, 4 per workgroup, grid-stride beyond
    // 4096 workgroups (the list's length is only known on the device)
    int64_t g = (a.tcap + 3) / 4;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
#define DG_CASE(NV_, K_)                                                                          \
    if (nv == NV_ && k == K_) {                                                                   \
        if (a.pk)                                                                                 \
            hipLaunchKernelGGL((blend2d_kernel<K_, NV_, TB, (K_ > 0)>), dim3((unsigned)g), dim3(256), 0, \
                               st, a.out, a.tcount, a.tcell, a.tdata, a.eta_acc, a.ctrl,          \
                               a.dt_from_ctrl, (long long)a.tcap, pp, a.pcount, a.pcell, a.pcap); \
        else                                                                                      \
            hipLaunchKernelGGL((blend2d_kernel<K_, NV_, TB, false>), dim3((unsigned)g), dim3(256), 0, \
                               st, a.out, a.tcount, a.tcell, a.tdata, a.eta_acc, a.ctrl,          \
                               a.dt_from_ctrl, (long long)a.tcap, pp, a.pcount, a.pcell, a.pcap); \
        return hipGetLastError();                                                                 \
    }
    DG_CASE(1, 0) DG_CASE(1, 1) DG_CASE(1, 2) DG_CASE(1, 3)
    DG_CASE(4, 0) DG_CASE(4, 1) DG_CASE(4, 2) DG_CASE(4, 3)
#undef DG_CASE
    return hipErrorInvalidValue;
}

template <typename TB>
hipError_t launch_pp2d(int k, StateView<TB> u, int64_t ncell, const unsigned long long* count,
                       const long long* cells, int64_t cap, const Ctrl* ctrl, int from_ctrl, int pk,
                       PPArgs pp, hipStream_t st)
{
    // one wavefront per cell, 4 per workgroup, grid-stride beyond 4096
    // workgroups
    const int64_t span = count ? cap : ncell;
    int64_t g = (span + 3) / 4;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
#define DG_CASE(K_)                                                                                \
    if (k == K_) {                                                                                 \
        if (pk)                                                                                    \
            hipLaunchKernelGGL((pp2d_kernel<K_, TB, (K_ > 0)>), dim3((unsigned)g), dim3(256), 0, st, u, \
                               (long long)ncell, count, cells, (long long)cap, ctrl, from_ctrl, pp); \
        else                                                                                       \
            hipLaunchKernelGGL((pp2d_kernel<K_, TB, false>), dim3((unsigned)g), dim3(256), 0, st, u,  \
                               (long long)ncell, count, cells, (long long)cap, ctrl, from_ctrl, pp); \
        return hipGetLastError();                                                                  \
    }
    DG_CASE(0) DG_CASE(1) DG_CASE(2) DG_CASE(3)
#undef DG_CASE
    return hipErrorInvalidValue;
}

template <typename TB>
hipError_t launch_maxwave2d(int eq, StateView<TB> u, int64_t nx, int64_t ny, double inv_hx,
                            double inv_hy, PhysParams phys, unsigned long long* acc, Ctrl* err,
                            hipStream_t st)
{
    const int64_t n = nx * ny;
    dim3 grid((unsigned)((n + 255) / 256)), block(256);
    if (eq == ADV)
        hipLaunchKernelGGL((maxwave2d_kernel<ADV, TB>), grid, block, 0, st, u, n, inv_hx, inv_hy, phys,
                           acc, err);
    else
        hipLaunchKernelGGL((maxwave2d_kernel<EULER, TB>), grid, block, 0, st, u, n, inv_hx, inv_hy,
                           phys, acc, err);
    return hipGetLastError();
}

#define DG_INST(TB)                                                                               \
    template hipError_t launch_stage2d<TB>(int, int, const Args2D<TB>&, hipStream_t);             \
    template hipError_t launch_filter2d<TB>(int, int, const Args2D<TB>&, hipStream_t);           \
    template hipError_t launch_indicator2d<TB>(int, int, const Args2D<TB>&, hipStream_t);       \
    template hipError_t launch_troubled2d<TB>(int, int, const Args2D<TB>&, hipStream_t);         \
    template hipError_t launch_blend2d<TB>(int, int, const Args2D<TB>&, PPArgs, hipStream_t);    \
    template hipError_t launch_pp2d<TB>(int, StateView<TB>, int64_t, const unsigned long long*,  \
                                        const long long*, int64_t, const Ctrl*, int, int, PPArgs,\
                                        hipStream_t);                                            \
    template hipError_t launch_convert_pk2d<TB>(int, int, int, int64_t, const double*,           \
                                                StateView<TB>, hipStream_t);                      \
    template hipError_t launch_maxwave2d<TB>(int, StateView<TB>, int64_t, int64_t, double, double, \
                                             PhysParams, unsigned long long*, Ctrl*, hipStream_t);
DG_INST(double)
DG_INST(float)
#undef DG_INST

}  // namespace dg
