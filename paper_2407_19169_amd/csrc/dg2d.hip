// dg2d.hip — 2D Q^k RKDG stage, jump filter, hybrid limiter and CFL
// kernels for gfx950 (arXiv:2407.19169, Sec. 2.3 two-dimensional scheme and
// filter, Sec. 2.4 systems, Sec. 3 Algorithm 1).
//
// Mapping: 16x16 cells per 256-thread workgroup, one thread per cell,
// x-fastest SoA mode planes (each plane load is a coalesced row access).
// The LDS tile has an 18x18 slot grid: the 16x16 own cells plus a ring of 64
// neighbours, filled by global cell coordinate (wrapped when periodic,
// flagged when outside the domain), so ragged tiles need no special case.
//   stage2d:  traces of each cell's right/top edges (and the ring's facing
//             edges) go to LDS; each edge flux is evaluated once per tile at
//             the Q Gauss points of the edge; the LDS is then reused for the
//             fluxes; volume quadrature by partial sum factorisation.
//   filter2d: one variable at a time, the modes of the tile + ring are staged
//             in LDS; the jumps of every mixed derivative at the two corners
//             of each edge are sum-factorised contractions of the two cells'
//             modes with the derivative values P_p^(a)(+-1).
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
        const T ir = (T)1 / u[0];
        const T vx = u[1] * ir, vy = u[2] * ir;
        const T pr = ((T)p.gamma - (T)1) * (u[3] - (T)0.5 * (u[1] * vx + u[2] * vy));
        const T vn = dir == 0 ? vx : vy;
        f[0] = u[0] * vn;
        f[1] = u[1] * vn + (dir == 0 ? pr : (T)0);
        f[2] = u[2] * vn + (dir == 1 ? pr : (T)0);
        f[3] = vn * (u[3] + pr);
    }
    template <typename T>
    __device__ static T speed(const T* u, int dir, const PhysParams& p)
    {
        const T pr = pressure(u, p);
        return fabs(u[1 + dir] / u[0]) + tsqrt<T>((T)p.gamma * pr / u[0]);
    }
    template <typename T>
    __device__ static T enthalpy(const T* u, const PhysParams& p)
    {
        return (u[3] + pressure(u, p)) / u[0];
    }
};

template <int EQ, typename T>
__device__ __forceinline__ void llf2d(const T* ul, const T* ur, int dir, T* fh, const PhysParams& p)
{
    constexpr int NV = Phys2D<EQ>::NV;
    T fl[NV], fr[NV];
    Phys2D<EQ>::flux(ul, dir, fl, p);
    Phys2D<EQ>::flux(ur, dir, fr, p);
    const T al = Phys2D<EQ>::speed(ul, dir, p), ar = Phys2D<EQ>::speed(ur, dir, p);
    const T alpha = al > ar ? al : ar;
#pragma unroll
    for (int v = 0; v < NV; ++v) fh[v] = (T)0.5 * (fl[v] + fr[v]) - (T)0.5 * alpha * (ur[v] - ul[v]);
}

// Global index along an axis: wrapped if periodic, -1 if outside.
__device__ __forceinline__ int64_t slot_index(int64_t g, int64_t n, bool periodic)
{
    if (g >= 0 && g < n) return g;
    if (!periodic) return -1;
    int64_t r = g % n;
    return r < 0 ? r + n : r;
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

// modes of one cell: u0 (FP64 mode 0) and uh[v][m-1] for m = p*K1+q >= 1
template <int NV, int NM, typename TB>
__device__ __forceinline__ void load_cell2d(const StateView<TB>& s, int64_t c, double (&u0)[NV],
                                            TB (&uh)[NV][NM > 1 ? NM - 1 : 1])
{
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        u0[v] = s.m0[v * s.s0 + c];
#pragma unroll
        for (int m = 1; m < NM; ++m) uh[v][m - 1] = s.hi[v * s.sv + (m - 1) * s.sl + c];
    }
}

// P_l^(m)(+-1) as a compile-time constant: side 0 -> -1, side 1 -> +1
__device__ __forceinline__ constexpr double dtr(int l, int m, int side)
{
    return side ? dtrace_r(l, m) : dtrace_l(l, m);
}

// Values of a cell's polynomial at the Q Gauss points of one face (FACE 0
// left xi=-1, 1 right xi=+1, 2 bottom eta=-1, 3 top eta=+1): first the sum
// across the face, then the along-face Legendre series.  Own cells and the
// tile's ring cells both use this routine, so the two workgroups that
// evaluate a tile-boundary edge flux see bitwise identical traces (the
// FP64 mode-0 update then telescopes exactly).
template <int FACE, int NV, int K, typename TB, typename T>
__device__ __forceinline__ void face_trace(const double (&u0)[NV],
                                           const TB (&uh)[NV][(K + 1) * (K + 1) > 1 ? (K + 1) * (K + 1) - 1 : 1],
                                           T (&tr)[K + 1][NV])
{
    constexpr int K1 = K + 1;
    constexpr bool xface = FACE < 2;
    constexpr bool plus = (FACE & 1) != 0;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        T c[K1];
#pragma unroll
        for (int o = 0; o < K1; ++o) {
            T s = (T)0;
#pragma unroll
            for (int n = 0; n < K1; ++n) {
                const int p = xface ? n : o, q = xface ? o : n;
                const T val = (p == 0 && q == 0) ? (T)u0[v] : (T)uh[v][p * K1 + q - 1];
                s += (plus || !(n & 1)) ? val : -val;
            }
            c[o] = s;
        }
#pragma unroll
        for (int b = 0; b < K1; ++b) {
            T s = (T)0;
#pragma unroll
            for (int o = 0; o < K1; ++o) s += c[o] * (T)leg_at(K1, b, o);
            tr[b][v] = s;
        }
    }
}

}  // namespace

template <int EQ, int K, typename TB>
__device__ __forceinline__ double stage2d_own_cell(const Args2D<TB>& a, int tid, int tx, int ty,
                                                   int64_t ix, int64_t jy, int stage, double dt,
                                                   const double (&u0)[Phys2D<EQ>::NV],
                                                   const TB (&uh)[Phys2D<EQ>::NV][(K + 1) * (K + 1) > 1 ? (K + 1) * (K + 1) - 1 : 1],
                                                   const TB* sFx, const TB* sFy);

// -------------------------------------------------------------------------
// Residual + Shu-Osher combination (no filter) -> a.out.  With alpha_acc the
// kernel accumulates the CFL quantity max(lambda_x/hx + lambda_y/hy) of its
// output's cell averages.
// -------------------------------------------------------------------------
template <int EQ, int K, typename TB>
__global__ __launch_bounds__(256) void stage2d_kernel(Args2D<TB> a)
{
    using P = Phys2D<EQ>;
    using T = TB;
    constexpr int NV = P::NV, K1 = K + 1, NM = K1 * K1, Q = K1, NH = NM > 1 ? NM - 1 : 1;
    constexpr int TS = Q * NV;                       // values of one edge trace / flux
    constexpr int NTR = 17 * 16 + 16 + 16 * 17 + 16;  // trace slots
    constexpr int NFL = 16 * 17 + 17 * 16;           // flux slots
    __shared__ __align__(16) T lds[(NTR > NFL ? NTR : NFL) * TS];

    if (a.dt_from_ctrl && a.ctrl->done) return;
    const double dt = a.dt_from_ctrl ? a.ctrl->dt : a.dt_host;
    const double t0 = a.dt_from_ctrl ? a.ctrl->t : a.t_host;
    const int stage = a.stage;
    const double ts = t0 + (stage == 0 ? 0.0 : stage == 1 ? dt : 0.5 * dt);

    // trace regions: R[ty][0..16] right traces of slot cols 0..16, Lr[ty]
    // left trace of slot col 17, Tt[tx][0..16] top traces of slot rows 0..16,
    // Br[tx] bottom trace of slot row 17.
    T* sR = lds;
    T* sLr = sR + 16 * 17 * TS;
    T* sT = sLr + 16 * TS;
    T* sBr = sT + 16 * 17 * TS;
    // flux regions (after the traces are consumed): Fx[ty][e], e = 0..16 the
    // vertical edges of row ty; Fy[tx][e] the horizontal edges of column tx.
    T* sFx = lds;
    T* sFy = lds + 16 * 17 * TS;

    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    const int64_t ix0 = (int64_t)blockIdx.x * 16, jy0 = (int64_t)blockIdx.y * 16;
    const int64_t ix = ix0 + tx, jy = jy0 + ty;
    const bool px = a.bc[0] == BC_PERIODIC, py = a.bc[2] == BC_PERIODIC;
    const int64_t cx = slot_index(ix, a.nx, px), cy = slot_index(jy, a.ny, py);
    const bool loadable = cx >= 0 && cy >= 0;
    const bool own = ix < a.nx && jy < a.ny;

    double u0[NV];
    T uh[NV][NH];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        u0[v] = 0.0;
#pragma unroll
        for (int m = 0; m < NH; ++m) uh[v][m] = (T)0;
    }
    if (loadable) load_cell2d<NV, NM, TB>(a.us, cy * a.nx + cx, u0, uh);
    auto mode = [&](int v, int p, int q) -> T {
        return (p == 0 && q == 0) ? (T)u0[v] : uh[v][p * K1 + q - 1];
    };

    // Edge traces at the Gauss points: u(+-1, eta_b) and u(xi_a, +-1).
    T trL[Q][NV], trR[Q][NV], trB[Q][NV], trT[Q][NV];
    face_trace<0, NV, K, TB, T>(u0, uh, trL);
    face_trace<1, NV, K, TB, T>(u0, uh, trR);
    face_trace<2, NV, K, TB, T>(u0, uh, trB);
    face_trace<3, NV, K, TB, T>(u0, uh, trT);
    (void)mode;
#pragma unroll
    for (int b = 0; b < Q; ++b)
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            sR[(ty * 17 + tx + 1) * TS + b * NV + v] = trR[b][v];
            sT[(tx * 17 + ty + 1) * TS + b * NV + v] = trT[b][v];
        }

    // Ring: 64 threads each load one neighbour cell of the tile and publish
    // the trace of its edge that faces the tile.
    if (tid < 64) {
        const int g = tid >> 4, i = tid & 15;
        const int64_t gx = g == 0 ? ix0 - 1 : g == 1 ? ix0 + 16 : ix0 + i;
        const int64_t gy = g == 2 ? jy0 - 1 : g == 3 ? jy0 + 16 : jy0 + i;
        const int64_t hx_ = slot_index(gx, a.nx, px), hy_ = slot_index(gy, a.ny, py);
        if (hx_ >= 0 && hy_ >= 0) {
            double w0[NV];
            T wh[NV][NH];
            load_cell2d<NV, NM, TB>(a.us, hy_ * a.nx + hx_, w0, wh);
            // the face of the ring cell that faces the tile: g=0 right, 1 left,
            // 2 top, 3 bottom
            T* dst = g == 0 ? &sR[(i * 17 + 0) * TS]
                   : g == 1 ? &sLr[i * TS]
                   : g == 2 ? &sT[(i * 17 + 0) * TS]
                            : &sBr[i * TS];
            T tr[Q][NV];
            if (g == 0)
                face_trace<1, NV, K, TB, T>(w0, wh, tr);
            else if (g == 1)
                face_trace<0, NV, K, TB, T>(w0, wh, tr);
            else if (g == 2)
                face_trace<3, NV, K, TB, T>(w0, wh, tr);
            else
                face_trace<2, NV, K, TB, T>(w0, wh, tr);
#pragma unroll
            for (int b = 0; b < Q; ++b)
#pragma unroll
                for (int v = 0; v < NV; ++v) dst[b * NV + v] = tr[b][v];
        }
    }
    __syncthreads();

    // Edge fluxes (LLF, normal +x / +y) at the Gauss points of the edges.
    T fLx[Q][NV], fBy[Q][NV], fRx[Q][NV], fTy[Q][NV];
    const bool need_r = loadable && (tx == 15 || (!px && ix == a.nx - 1));
    const bool need_t = loadable && (ty == 15 || (!py && jy == a.ny - 1));
    if (loadable) {
        const bool lghost = !px && ix == 0, bghost = !py && jy == 0;
        const bool rghost = !px && ix == a.nx - 1, tghost = !py && jy == a.ny - 1;
        const double xl = a.xlo + (double)ix * a.hx, yb = a.ylo + (double)jy * a.hy;
#pragma unroll
        for (int b = 0; b < Q; ++b) {
            const double yq = yb + 0.5 * a.hy * (1.0 + gl_node(Q, b));
            const double xq = xl + 0.5 * a.hx * (1.0 + gl_node(Q, b));
            T left[NV], bot[NV];
            if (lghost)
                ghost_state2d<NV, TB, T>(a, 0, xl, yq, ts, trL[b], left);
            else
#pragma unroll
                for (int v = 0; v < NV; ++v) left[v] = sR[(ty * 17 + tx) * TS + b * NV + v];
            llf2d<EQ, T>(left, trL[b], 0, fLx[b], a.phys);
            if (bghost)
                ghost_state2d<NV, TB, T>(a, 2, xq, yb, ts, trB[b], bot);
            else
#pragma unroll
                for (int v = 0; v < NV; ++v) bot[v] = sT[(tx * 17 + ty) * TS + b * NV + v];
            llf2d<EQ, T>(bot, trB[b], 1, fBy[b], a.phys);
            if (need_r) {
                T right[NV];
                if (rghost)
                    ghost_state2d<NV, TB, T>(a, 1, xl + a.hx, yq, ts, trR[b], right);
                else
#pragma unroll
                    for (int v = 0; v < NV; ++v) right[v] = sLr[ty * TS + b * NV + v];
                llf2d<EQ, T>(trR[b], right, 0, fRx[b], a.phys);
            }
            if (need_t) {
                T top[NV];
                if (tghost)
                    ghost_state2d<NV, TB, T>(a, 3, xq, yb + a.hy, ts, trT[b], top);
                else
#pragma unroll
                    for (int v = 0; v < NV; ++v) top[v] = sBr[tx * TS + b * NV + v];
                llf2d<EQ, T>(trT[b], top, 1, fTy[b], a.phys);
            }
        }
    }
    __syncthreads();  // traces consumed; reuse the LDS for the fluxes
    if (loadable) {
#pragma unroll
        for (int b = 0; b < Q; ++b)
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                sFx[(ty * 17 + tx) * TS + b * NV + v] = fLx[b][v];
                sFy[(tx * 17 + ty) * TS + b * NV + v] = fBy[b][v];
                if (need_r) sFx[(ty * 17 + tx + 1) * TS + b * NV + v] = fRx[b][v];
                if (need_t) sFy[(tx * 17 + ty + 1) * TS + b * NV + v] = fTy[b][v];
            }
    }
    __syncthreads();

    double lam_out = 0.0;
    if (own) lam_out = stage2d_own_cell<EQ, K, TB>(a, tid, tx, ty, ix, jy, stage, dt, u0, uh, sFx, sFy);
    // every lane reaches the wave reduction (no early exits above)
    if (a.alpha_acc) {
        const double z = wave_max(lam_out);
        if ((tid & 63) == 0) atomic_max_nonneg(a.alpha_acc, z);
    }
}

// Volume term, edge terms, residual and Shu-Osher combination of one own
// cell (the fluxes of its four edges are in LDS); returns the CFL quantity
// lambda_x/hx + lambda_y/hy of the output's cell average.
template <int EQ, int K, typename TB>
__device__ __forceinline__ double stage2d_own_cell(const Args2D<TB>& a, int tid, int tx, int ty,
                                                   int64_t ix, int64_t jy, int stage, double dt,
                                                   const double (&u0)[Phys2D<EQ>::NV],
                                                   const TB (&uh)[Phys2D<EQ>::NV][(K + 1) * (K + 1) > 1 ? (K + 1) * (K + 1) - 1 : 1],
                                                   const TB* sFx, const TB* sFy)
{
    using P = Phys2D<EQ>;
    using T = TB;
    constexpr int NV = P::NV, K1 = K + 1, NM = K1 * K1, Q = K1, NH = NM > 1 ? NM - 1 : 1;
    constexpr int TS = Q * NV;
    auto mode = [&](int v, int p, int q) -> T {
        return (p == 0 && q == 0) ? (T)u0[v] : uh[v][p * K1 + q - 1];
    };
    const int64_t cell = jy * a.nx + ix;

    // Volume term: (hy/2) sum w_a w_b F1 P_p'(xi_a) P_q(eta_b)
    //            + (hx/2) sum w_a w_b F2 P_p(xi_a) P_q'(eta_b)
    T acc[NV][NM];
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int m = 0; m < NM; ++m) acc[v][m] = (T)0;
    const T hy2 = (T)(0.5 * a.hy), hx2 = (T)(0.5 * a.hx);
#pragma unroll
    for (int qa = 0; qa < Q; ++qa) {
        T col[NV][K1];  // sum_p u^{pq} P_p(xi_a)
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int q = 0; q < K1; ++q) {
                T s = (T)0;
#pragma unroll
                for (int p = 0; p < K1; ++p) s += mode(v, p, q) * (T)leg_at(Q, qa, p);
                col[v][q] = s;
            }
        T t1[NV][K1], t2[NV][K1];  // sum_b w_b F1 P_q(eta_b), sum_b w_b F2 P_q'(eta_b)
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int q = 0; q < K1; ++q) t1[v][q] = t2[v][q] = (T)0;
#pragma unroll
        for (int qb = 0; qb < Q; ++qb) {
            T uq[NV], f1[NV], f2[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                T s = (T)0;
#pragma unroll
                for (int q = 0; q < K1; ++q) s += col[v][q] * (T)leg_at(Q, qb, q);
                uq[v] = s;
            }
            if (EQ == EULER && a.check) {
                const T pr = Phys2D<EULER>::pressure(uq, a.phys);
                if (!(uq[0] > (T)0) || !(pr > (T)0)) {
                    const bool fin = isfinite((double)uq[0]) && isfinite((double)pr);
                    latch_error(a.ctrl, fin ? -5 : -4, cell);
                }
            }
            P::flux(uq, 0, f1, a.phys);
            P::flux(uq, 1, f2, a.phys);
            const T wb = (T)gl_weight(Q, qb);
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int q = 0; q < K1; ++q) {
                    t1[v][q] += wb * f1[v] * (T)leg_at(Q, qb, q);
                    t2[v][q] += wb * f2[v] * (T)dleg_at(Q, qb, q);
                }
        }
        const T wa = (T)gl_weight(Q, qa);
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int p = 0; p < K1; ++p)
#pragma unroll
                for (int q = 0; q < K1; ++q)
                    acc[v][p * K1 + q] += wa * (hy2 * (T)dleg_at(Q, qa, p) * t1[v][q] +
                                                hx2 * (T)leg_at(Q, qa, p) * t2[v][q]);
    }

    // Edge terms, residual, Shu-Osher combination.
    double n0[NV];
    T nh[NV][NH];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        n0[v] = 0.0;
#pragma unroll
        for (int m = 0; m < NH; ++m) nh[v][m] = (T)0;
    }
    if (stage > 0) load_cell2d<NV, NM, TB>(a.un, cell, n0, nh);
    const T* FL = &sFx[(ty * 17 + tx) * TS];
    const T* FR = &sFx[(ty * 17 + tx + 1) * TS];
    const T* FB = &sFy[(tx * 17 + ty) * TS];
    const T* FT = &sFy[(tx * 17 + ty + 1) * TS];
    const double ivol = a.inv_hx * a.inv_hy;
    double v0[NV];
    T vh[NV][NH];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        // mode (0,0): -(hy/2) sum_b w_b (FR - FL) - (hx/2) sum_a w_a (FT - FB), in FP64
        double ex = 0.0, ey = 0.0;
#pragma unroll
        for (int b = 0; b < Q; ++b) {
            ex += gl_weight(Q, b) * ((double)FR[b * NV + v] - (double)FL[b * NV + v]);
            ey += gl_weight(Q, b) * ((double)FT[b * NV + v] - (double)FB[b * NV + v]);
        }
        const double L0 = -(0.5 * a.hy * ex + 0.5 * a.hx * ey) * ivol;
        v0[v] = combine2(stage, n0[v], u0[v] + dt * L0);
#pragma unroll
        for (int p = 0; p < K1; ++p)
#pragma unroll
            for (int q = 0; q < K1; ++q) {
                if (p == 0 && q == 0) continue;
                T ex_ = (T)0, ey_ = (T)0;
#pragma unroll
                for (int b = 0; b < Q; ++b) {
                    const T fl = (p & 1) ? -FL[b * NV + v] : FL[b * NV + v];
                    ex_ += (T)gl_weight(Q, b) * (FR[b * NV + v] - fl) * (T)leg_at(Q, b, q);
                    const T fb = (q & 1) ? -FB[b * NV + v] : FB[b * NV + v];
                    ey_ += (T)gl_weight(Q, b) * (FT[b * NV + v] - fb) * (T)leg_at(Q, b, p);
                }
                const T r = acc[v][p * K1 + q] - hy2 * ex_ - hx2 * ey_;
                const T L = (T)((2 * p + 1) * (2 * q + 1)) * (T)ivol * r;
                const int m = p * K1 + q - 1;
                vh[v][m] = combine2_t<T>(stage, nh[v][m], uh[v][m] + (T)dt * L);
            }
    }
    // store
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        a.out.m0[v * a.out.s0 + cell] = v0[v];
#pragma unroll
        for (int m = 1; m < NM; ++m) a.out.hi[v * a.out.sv + (m - 1) * a.out.sl + cell] = vh[v][m - 1];
    }
    (void)tid;
    return P::speed(v0, 0, a.phys) * a.inv_hx + P::speed(v0, 1, a.phys) * a.inv_hy;
}

// -------------------------------------------------------------------------
// Jump filter (MODE 1: filtered copy of a.us into a.out) or hybrid pass A
// (MODE 2: records of the troubled cells of a.us, and max eta).
//   E^l = dt / (hx hy H) * max_v [hx beta_x Sx^l_v + hy beta_y Sy^l_v],
//   Sx^l = sum_{|a| <= l} jsx[a] * Jx^a (edge-averaged |[d^a u]| in reference
//   derivatives; jsx[0] = hx, jsx[a] = m(m+1) hx^(m+1) (2/hx)^a1 (2/hy)^a2).
// -------------------------------------------------------------------------
template <int EQ, int K, typename TB, int MODE>
__global__ __launch_bounds__(256) void filter2d_kernel(Args2D<TB> a)
{
    using P = Phys2D<EQ>;
    using T = TB;
    constexpr int NV = P::NV, K1 = K + 1, NM = K1 * K1, L1 = 2 * K + 1;
    __shared__ __align__(16) T sM[18 * 18 * NM];

    if (a.dt_from_ctrl && a.ctrl->done) return;
    const double dt = a.dt_from_ctrl ? a.ctrl->dt : a.dt_host;
    const double t0 = a.dt_from_ctrl ? a.ctrl->t : a.t_host;
    const double tf = t0 + (a.stage == 1 ? 0.5 : 1.0) * dt;  // time the stage output stands for

    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    const int64_t ix0 = (int64_t)blockIdx.x * 16, jy0 = (int64_t)blockIdx.y * 16;
    const int64_t ix = ix0 + tx, jy = jy0 + ty;
    const bool px = a.bc[0] == BC_PERIODIC, py = a.bc[2] == BC_PERIODIC;
    const int64_t cx = slot_index(ix, a.nx, px), cy = slot_index(jy, a.ny, py);
    const bool loadable = cx >= 0 && cy >= 0;
    const bool own = ix < a.nx && jy < a.ny;
    // ring slot of this thread (tid < 64)
    const int g = tid >> 4, gi = tid & 15;
    const int64_t rgx = g == 0 ? ix0 - 1 : g == 1 ? ix0 + 16 : ix0 + gi;
    const int64_t rgy = g == 2 ? jy0 - 1 : g == 3 ? jy0 + 16 : jy0 + gi;
    const int64_t rcx = slot_index(rgx, a.nx, px), rcy = slot_index(rgy, a.ny, py);
    const int rslot = g == 0 ? (gi + 1) * 18 + 0 : g == 1 ? (gi + 1) * 18 + 17 : g == 2 ? 0 * 18 + gi + 1
                                                                                        : 17 * 18 + gi + 1;
    const int oslot = (ty + 1) * 18 + tx + 1;
    const bool lin = slot_index(ix - 1, a.nx, px) >= 0, rin = slot_index(ix + 1, a.nx, px) >= 0;
    const bool bin = slot_index(jy - 1, a.ny, py) >= 0, tin = slot_index(jy + 1, a.ny, py) >= 0;
    const double xl = a.xlo + (double)ix * a.hx, yb = a.ylo + (double)jy * a.hy;

    T best[L1];
#pragma unroll
    for (int l = 0; l < L1; ++l) best[l] = (T)0;
    T eta = (T)0;
    double ub[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) ub[v] = loadable ? a.us.m0[v * a.us.s0 + cy * a.nx + cx] : 1.0;
    T ubt[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) ubt[v] = (T)ub[v];
    const T bx = P::speed(ubt, 0, a.phys), by = P::speed(ubt, 1, a.phys);
    const T H = P::enthalpy(ubt, a.phys);

    for (int v = 0; v < NV; ++v) {
        __syncthreads();
        if (loadable) {
            const int64_t c = cy * a.nx + cx;
            sM[oslot * NM] = (T)a.us.m0[v * a.us.s0 + c];
#pragma unroll
            for (int m = 1; m < NM; ++m) sM[oslot * NM + m] = a.us.hi[v * a.us.sv + (m - 1) * a.us.sl + c];
        }
        if (tid < 64 && rcx >= 0 && rcy >= 0) {
            const int64_t c = rcy * a.nx + rcx;
            sM[rslot * NM] = (T)a.us.m0[v * a.us.s0 + c];
#pragma unroll
            for (int m = 1; m < NM; ++m) sM[rslot * NM + m] = a.us.hi[v * a.us.sv + (m - 1) * a.us.sl + c];
        }
        __syncthreads();
        if (!own) continue;
        const T* U0 = &sM[oslot * NM];
        T Jx[L1], Jy[L1];  // weighted sums per derivative order m = a1 + a2
#pragma unroll
        for (int m = 0; m < L1; ++m) Jx[m] = Jy[m] = (T)0;
        T jx0 = (T)0, jy0_ = (T)0;
        // vertical faces: side 0 (left, neighbour slot -1) and 1 (right, +1)
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const bool inside = side ? rin : lin;
            const T* UN = &sM[(oslot + (side ? 1 : -1)) * NM];
            // G[a1][q] = sum_p u^{pq} P_p^(a1)(end): own at its `side` end,
            // neighbour at the opposite end
            T D[K1][K1];  // D[a1][q] = G_nb - G_own (or G_own if ghost)
#pragma unroll
            for (int a1 = 0; a1 < K1; ++a1)
#pragma unroll
                for (int q = 0; q < K1; ++q) {
                    T go = (T)0, gn = (T)0;
#pragma unroll
                    for (int p = (a1 > 0 ? a1 : 0); p < K1; ++p) {
                        go += U0[p * K1 + q] * (T)dtr(p, a1, side);
                        if (inside) gn += UN[p * K1 + q] * (T)dtr(p, a1, 1 - side);
                    }
                    D[a1][q] = inside ? gn - go : go;
                }
            const double xf = xl + (side ? a.hx : 0.0);
#pragma unroll
            for (int cyc = 0; cyc < 2; ++cyc) {
                const double yc = yb + (cyc ? a.hy : 0.0);
#pragma unroll
                for (int a1 = 0; a1 < K1; ++a1)
#pragma unroll
                    for (int a2 = 0; a2 < K1; ++a2) {
                        T s = (T)0;
#pragma unroll
                        for (int q = (a2 > 0 ? a2 : 0); q < K1; ++q) s += D[a1][q] * (T)dtr(q, a2, cyc);
                        T j = inside ? fabs(s) : ghost_jump2d<TB, T>(a, side, xf, yc, tf, a1, a2, v, s);
                        Jx[a1 + a2] += (T)(0.5 * a.jsx[a1 * 4 + a2]) * j;
                        if (a1 == 0 && a2 == 0) jx0 += (T)0.5 * j;
                    }
            }
        }
        // horizontal faces: side 0 (bottom, slot -18) and 1 (top, +18)
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const bool inside = side ? tin : bin;
            const T* UN = &sM[(oslot + (side ? 18 : -18)) * NM];
            T D[K1][K1];  // D[p][a2]
#pragma unroll
            for (int p = 0; p < K1; ++p)
#pragma unroll
                for (int a2 = 0; a2 < K1; ++a2) {
                    T go = (T)0, gn = (T)0;
#pragma unroll
                    for (int q = (a2 > 0 ? a2 : 0); q < K1; ++q) {
                        go += U0[p * K1 + q] * (T)dtr(q, a2, side);
                        if (inside) gn += UN[p * K1 + q] * (T)dtr(q, a2, 1 - side);
                    }
                    D[p][a2] = inside ? gn - go : go;
                }
            const double yf = yb + (side ? a.hy : 0.0);
#pragma unroll
            for (int cxc = 0; cxc < 2; ++cxc) {
                const double xc = xl + (cxc ? a.hx : 0.0);
#pragma unroll
                for (int a1 = 0; a1 < K1; ++a1)
#pragma unroll
                    for (int a2 = 0; a2 < K1; ++a2) {
                        T s = (T)0;
#pragma unroll
                        for (int p = (a1 > 0 ? a1 : 0); p < K1; ++p) s += D[p][a2] * (T)dtr(p, a1, cxc);
                        T j = inside ? fabs(s) : ghost_jump2d<TB, T>(a, 2 + side, xc, yf, tf, a1, a2, v, s);
                        Jy[a1 + a2] += (T)(0.5 * a.jsy[a1 * 4 + a2]) * j;
                        if (a1 == 0 && a2 == 0) jy0_ += (T)0.5 * j;
                    }
            }
        }
        // running partial sums over the derivative order and max over vars
        T sx = (T)0, sy = (T)0;
#pragma unroll
        for (int l = 0; l < L1; ++l) {
            sx += Jx[l];
            sy += Jy[l];
            const T sv = (T)a.cfmx * bx * sx + (T)a.cfmy * by * sy;
            best[l] = (v == 0 || sv > best[l]) ? sv : best[l];
        }
        const T ev = jx0 * (T)(0.5 * a.inv_hx) + jy0_ * (T)(0.5 * a.inv_hy);
        eta = (v == 0 || ev > eta) ? ev : eta;
    }
    if (MODE == 2) {
        // max eta over the grid: every lane reaches the wave reduction
        const double z = wave_max(own ? (double)eta : 0.0);
        if ((tid & 63) == 0) atomic_max_nonneg(a.eta_acc, z);
    }
    if (!own) return;
    const int64_t cell = jy * a.nx + ix;
    const T coef = (T)dt * (T)(a.inv_hx * a.inv_hy) / H;
    T E[L1];
    E[0] = (T)0;
#pragma unroll
    for (int l = 1; l < L1; ++l) E[l] = coef * best[l];
    if (a.E_out) {
#pragma unroll
        for (int l = 0; l < L1; ++l) a.E_out[cell * L1 + l] = (double)E[l];
    }
    if constexpr (MODE == 1) {
        T f[L1];
#pragma unroll
        for (int l = 1; l < L1; ++l) f[l] = texp<T>(-E[l]);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            a.out.m0[v * a.out.s0 + cell] = a.us.m0[v * a.us.s0 + cell];
#pragma unroll
            for (int p = 0; p < K1; ++p)
#pragma unroll
                for (int q = 0; q < K1; ++q) {
                    if (p == 0 && q == 0) continue;
                    const int m = p * K1 + q - 1;
                    a.out.hi[v * a.out.sv + m * a.out.sl + cell] = a.us.hi[v * a.us.sv + m * a.us.sl + cell] * f[p + q];
                }
        }
    } else {
        if (a.eta_out) a.eta_out[cell] = (double)eta;
        if (eta > (T)1) {
            const unsigned int slot = atomicAdd(a.tcount, 1u);
            if ((long long)slot < a.tcap) {
                a.tcell[slot] = cell;
                double* rec = a.tdata + (size_t)slot * L1;
                rec[0] = (double)eta;
#pragma unroll
                for (int l = 1; l < L1; ++l) rec[l] = (double)E[l];
            }
        }
    }
}

// Hybrid pass B over the troubled list: u^{pq} <- [w + (1 - w) exp(-E^{p+q})] u^{pq}.
template <int K, int NV, typename TB>
__global__ __launch_bounds__(256) void blend2d_kernel(StateView<TB> out, const unsigned int* count,
                                                      const long long* tcell, const double* tdata,
                                                      const unsigned long long* eta_bits,
                                                      const Ctrl* ctrl, int from_ctrl, long long cap)
{
    constexpr int K1 = K + 1, L1 = 2 * K + 1;
    if (from_ctrl && ctrl->done) return;
    unsigned int cnt = *count;
    if ((long long)cnt > cap) cnt = (unsigned int)cap;
    const double M = __longlong_as_double((long long)*eta_bits);
    for (unsigned int i = blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += gridDim.x * blockDim.x) {
        const long long c = tcell[i];
        const double* rec = tdata + (size_t)i * L1;
        const double w = (M - rec[0]) / (M - 1.0);
        TB f[L1];
#pragma unroll
        for (int l = 1; l < L1; ++l) f[l] = (TB)(w + (1.0 - w) * exp(-rec[l]));
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int p = 0; p < K1; ++p)
#pragma unroll
                for (int q = 0; q < K1; ++q) {
                    if (p == 0 && q == 0) continue;
                    out.hi[v * out.sv + (p * K1 + q - 1) * out.sl + c] *= f[p + q];
                }
    }
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
        lam = Phys2D<EQ>::speed(ub, 0, phys) * ihx + Phys2D<EQ>::speed(ub, 1, phys) * ihy;
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
    dim3 grid((unsigned)((a.nx + 15) / 16), (unsigned)((a.ny + 15) / 16)), block(256);
#define DG_CASE(E_, K_)                                                                   \
    if (eq == E_ && k == K_) {                                                            \
        hipLaunchKernelGGL((stage2d_kernel<E_, K_, TB>), grid, block, 0, st, a);          \
        return hipGetLastError();                                                         \
    }
    DG_CASE(ADV, 0) DG_CASE(ADV, 1) DG_CASE(ADV, 2) DG_CASE(ADV, 3)
    DG_CASE(EULER, 0) DG_CASE(EULER, 1) DG_CASE(EULER, 2) DG_CASE(EULER, 3)
#undef DG_CASE
    return hipErrorInvalidValue;
}

template <typename TB>
hipError_t launch_filter2d(int eq, int k, const Args2D<TB>& a, int mode, hipStream_t st)
{
    dim3 grid((unsigned)((a.nx + 15) / 16), (unsigned)((a.ny + 15) / 16)), block(256);
#define DG_CASE(E_, K_)                                                                        \
    if (eq == E_ && k == K_) {                                                                 \
        if (mode == 1)                                                                         \
            hipLaunchKernelGGL((filter2d_kernel<E_, K_, TB, 1>), grid, block, 0, st, a);       \
        else                                                                                   \
            hipLaunchKernelGGL((filter2d_kernel<E_, K_, TB, 2>), grid, block, 0, st, a);       \
        return hipGetLastError();                                                              \
    }
    DG_CASE(ADV, 0) DG_CASE(ADV, 1) DG_CASE(ADV, 2) DG_CASE(ADV, 3)
    DG_CASE(EULER, 0) DG_CASE(EULER, 1) DG_CASE(EULER, 2) DG_CASE(EULER, 3)
#undef DG_CASE
    return hipErrorInvalidValue;
}

template <typename TB>
hipError_t launch_blend2d(int nv, int k, StateView<TB> out, int64_t ncell, const unsigned int* count,
                          const long long* tcell, const double* tdata,
                          const unsigned long long* eta_bits, const Ctrl* ctrl, int from_ctrl,
                          int64_t max_entries, hipStream_t st)
{
    unsigned g = (unsigned)((max_entries + 255) / 256);
    if (g > 2048) g = 2048;
    if (g < 1) g = 1;
#define DG_CASE(NV_, K_)                                                                          \
    if (nv == NV_ && k == K_) {                                                                   \
        hipLaunchKernelGGL((blend2d_kernel<K_, NV_, TB>), dim3(g), dim3(256), 0, st, out, count,  \
                           tcell, tdata, eta_bits, ctrl, from_ctrl, (long long)max_entries);      \
        return hipGetLastError();                                                                 \
    }
    DG_CASE(1, 0) DG_CASE(1, 1) DG_CASE(1, 2) DG_CASE(1, 3)
    DG_CASE(4, 0) DG_CASE(4, 1) DG_CASE(4, 2) DG_CASE(4, 3)
#undef DG_CASE
    (void)ncell;
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
    template hipError_t launch_filter2d<TB>(int, int, const Args2D<TB>&, int, hipStream_t);       \
    template hipError_t launch_blend2d<TB>(int, int, StateView<TB>, int64_t, const unsigned int*, \
                                           const long long*, const double*,                      \
                                           const unsigned long long*, const Ctrl*, int, int64_t, \
                                           hipStream_t);                                         \
    template hipError_t launch_maxwave2d<TB>(int, StateView<TB>, int64_t, int64_t, double, double, \
                                             PhysParams, unsigned long long*, Ctrl*, hipStream_t);
DG_INST(double)
DG_INST(float)
#undef DG_INST

}  // namespace dg
