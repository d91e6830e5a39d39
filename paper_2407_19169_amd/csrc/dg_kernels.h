// dg_kernels.h — kernel argument blocks and launcher entry points of the
// RKDG + jump-filter library (internal; the public ABI is include/dg.h).
#pragma once

#include "dg_common.h"

namespace dg {

// SSP-RK3 effective quadrature weights of the three stage fluxes in the
// Shu-Osher form (1/6, 1/6, 2/3): the boundary-flux ledger uses them.
constexpr double kStageWeight[3] = {1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0};

template <typename TB>
struct Args1D {
    StateView<TB> un, us, out;
    int64_t n;
    double inv_h;
    int periodic, bc_lo, bc_hi;
    double dir_lo[4], dir_hi[4];
    PhysParams phys;
    int stage;
    int dt_from_ctrl;         // 1: dt and the done flag come from ctrl (dg_run)
    double dt_host;
    int check;                // Euler positivity check of the stage input
    Ctrl* ctrl;               // always valid: error latch
    int fold_ctrl;            // the last workgroup to finish runs the step control
                              // (MODE 2 single stage, n < kSmallTileCells)
    double* bflux;            // nullable: 8 doubles (x-lo[4], x-hi[4])
    unsigned long long* alpha_acc;  // nullable: CFL max of the output
    unsigned long long* eta_acc;    // hybrid
    unsigned int* tcount;           // hybrid pass A: troubled list
    long long* tcell;
    double* tdata;                  // (eta, E^1..E^k) per entry
    long long tcap;                 // capacity of the troubled list (entries)
    double* E_out;                  // nullable: per-cell exponents
    double* eta_out;                // per-cell eta (unfused hybrid)
    int want_lam;                   // return the CFL quantity without alpha_acc (batch)
    int pp;                         // Euler: positivity-preserving limiter after the filter
    int* reject;                    // pp: set when an output cell average is inadmissible
    // Hybrid with pass B deferred to the reader: pass A writes eta (every own
    // cell) and the exponents (troubled cells) per cell to dv_eta / dv_E
    // ([l-1][cell]); a stage that loads a state still owing its blend
    // applies it on load (bl_us for u^(s), bl_un for u^n).
    TB* dv_eta;                     // nullable
    TB* dv_E;
    struct Deferred {
        const TB* eta;              // nullable: no blend owed
        const TB* E;
        const unsigned long long* M;  // domain max of eta of that stage
    } bl_us, bl_un;
    unsigned long long* zero_bits;  // nullable: cleared by the first thread of the launch
};

// Positivity limiter inputs of the blend kernels (hybrid pass B and the
// per-call blend): the limiter runs after the blend.
struct PPArgs {
    int on;
    PhysParams phys;
    int* reject;                    // nullable: set on an inadmissible cell average
};

template <typename TB>
struct Args2D {
    StateView<TB> un, us, out;
    int64_t nx, ny;
    double hx, hy, inv_hx, inv_hy;
    double xlo, ylo;
    int bc[4];                // x-lo, x-hi, y-lo, y-hi
    double dir[4][4];         // Dirichlet states per side
    double shock_x0, shock_speed, post[4], pre[4];  // double-Mach boundaries
    PhysParams phys;
    int stage;
    int dt_from_ctrl;         // 1: dt, t and the done flag come from ctrl
    double dt_host, t_host;   // step size and step start time (per-call API)
    int check;
    Ctrl* ctrl;
    double* bflux;            // unused in 2D (periodic / open ledger via fluxes)
    unsigned long long* alpha_acc;
    unsigned long long* eta_acc;
    unsigned int* tcount;
    long long* tcell;
    double* tdata;            // (eta, E^1..E^{2k}) per entry
    long long tcap;
    double* E_out;            // nullable: per-cell exponents, (2k+1) per cell
    double* eta_out;
    double jsx[16], jsy[16];  // jump weights per multi-index a1*4+a2 (see filter2d)
    double cfmx, cfmy;        // mesh factors of (c_fx, c_fy) (cf_reading)
    int pk;                   // P^k space: compact planes of the modes p + q <= k
    // Euler positivity limiter: the post-stage kernels list the cells whose
    // screen fails (pcell, at most pcap, count in *pcount, cleared by the
    // stage kernel of the next stage), pp2d_kernel limits them
    int pp;
    unsigned long long* pcount;
    long long* pcell;
    long long pcap;
    int* reject;              // set when a limited cell's average is inadmissible
    // Hybrid runs: the stage kernel writes, and the indicator then reads, the
    // values of its output at the four cell corners, corner[(c NV + v)
    // cstride + cell] with c = sx + 2 sy (sx, sy = 1 at the +x, +y corner),
    // and with the positivity limiter its screen's verdict, ppfail[cell] = 1
    // when the screen does not clear the cell.  Null: the indicator reads
    // the state itself.
    TB* corner;
    unsigned char* ppfail;
    int64_t cstride;
};

template <typename TB>
hipError_t launch_stage2d(int eq, int k, const Args2D<TB>& a, hipStream_t st);
// The 2D jump filter, a.us -> a.out (and per-cell exponents to a.E_out if set).
template <typename TB>
hipError_t launch_filter2d(int eq, int k, const Args2D<TB>& a, hipStream_t st);
// Hybrid limiter in 2D (Algorithm 1) on a.us = a.out: pass A (the indicator
// of every cell, the domain maximum a.eta_acc, the troubled list a.tcount /
// tcell / tdata, the limiter's list), pass B1 (the exponents of the troubled
// cells into their tdata records, the state only read) and pass B2 (the
// blend of the troubled cells, then the limiter on them).
template <typename TB>
hipError_t launch_indicator2d(int eq, int k, const Args2D<TB>& a, hipStream_t st);
template <typename TB>
hipError_t launch_troubled2d(int eq, int k, const Args2D<TB>& a, hipStream_t st);
template <typename TB>
hipError_t launch_blend2d(int nv, int k, const Args2D<TB>& a, PPArgs pp, hipStream_t st);
// 2D Euler positivity limiter (Zhang and Shu on rectangles) in place on the
// cells listed by the post-stage kernels (count, cells; capacity cap), or on
// every cell when count is null.  Flags pp.reject when a cell average is
// inadmissible.
template <typename TB>
hipError_t launch_pp2d(int k, StateView<TB> u, int64_t ncell, const unsigned long long* count,
                       const long long* cells, int64_t cap, const Ctrl* ctrl, int from_ctrl, int pk,
                       PPArgs pp, hipStream_t st);
// FP64 exchange layout (every Q^k mode) <-> compact internal P^k planes
// (modes p + q <= k in p-major order); zeros for the other modes on the way out.
template <typename TB>
hipError_t launch_convert_pk2d(int to_internal, int nv, int k, int64_t ncell, const double* ext,
                               StateView<TB> v, hipStream_t st);
template <typename TB>
hipError_t launch_maxwave2d(int eq, StateView<TB> u, int64_t nx, int64_t ny, double inv_hx,
                            double inv_hy, PhysParams phys, unsigned long long* acc, Ctrl* err,
                            hipStream_t st);

template <typename TB>
// nst = 3 (MODE 0 or 1 only): the three SSP-RK3 stages of a step in one
// launch, u^n (a.un) -> u^{n+1} (a.out), intermediate stages in registers and
// LDS, boundary fluxes of stage s at a.bflux + 8 s.
hipError_t launch_stage1d(int eq, int k, const Args1D<TB>& a, int mode, hipStream_t st, int nst = 1);
template <typename TB>
hipError_t launch_filter1d(int eq, int k, const Args1D<TB>& a, int mode, hipStream_t st);
template <typename TB>
hipError_t launch_blend1d(int nv, int k, StateView<TB> out, const unsigned int* count,
                          const long long* tcell, const double* tdata,
                          const unsigned long long* eta_bits, const Ctrl* ctrl, int from_ctrl,
                          int64_t max_entries, PPArgs pp, hipStream_t st);
// The blend a state still owes (deferred hybrid pass B), applied in place.
template <typename TB>
hipError_t launch_deferred_blend1d(int nv, int k, StateView<TB> u, int64_t n,
                                   typename Args1D<TB>::Deferred bl, hipStream_t st);
template <typename TB>
hipError_t launch_blend_all1d(int nv, int k, StateView<TB> w, StateView<TB> out, int64_t n,
                              const double* E, const double* eta,
                              const unsigned long long* eta_bits, unsigned int* tcount,
                              PPArgs pp, hipStream_t st);
template <typename TB>
hipError_t launch_maxwave1d(int eq, StateView<TB> u, int64_t n, PhysParams phys,
                            unsigned long long* acc, Ctrl* err, hipStream_t st);

// Finalise the step that just ran (advance t, ledger, dt statistics) and,
// unless finalize_only, schedule the next one: dt = cfl_num / alpha from the
// CFL maximum accumulated by the previous step's last stage, clamped so the
// run ends exactly at t_end.  Called by one thread (step_ctrl_kernel).
template <typename C>
__device__ inline void step_ctrl_body(C* c, int finalize_only)
{
    if (finalize_only == 2) {  // clear the per-step accumulators only (and the
                               // arrival count: step_ctrl_kernel)
        c->alpha_bits = 0;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
            c->tcount[s] = 0;
            c->eta_line[s].v = 0;
        }
        return;
    }
    if (c->reject) {
        // positivity limiter: the step that just ran left an inadmissible
        // cell average; its output was replaced by u^n (restore kernel), so
        // it is run again with half the time step
        c->reject = 0;
        if (c->active && !c->done) {
            if (++c->retries > kMaxRetries) {
                if (c->status == 0) {
                    c->status = -5;
                    c->first_bad = -1;
                }
                c->active = 0;
                c->done = 1;
                return;
            }
            c->restarts += 1;
            c->dt *= 0.5;
            c->last = 0;
            c->alpha_bits = 0;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
                c->tcount[s] = 0;
                c->eta_line[s].v = 0;
#pragma unroll
        for (int v = 0; v < 8; ++v) c->bstage[s][v] = 0.0;
            }
            return;
        }
    }
    if (c->active) {
        c->retries = 0;
        const double dt = c->dt;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            double net = kStageWeight[0] * (c->bstage[0][4 + v] - c->bstage[0][v]) +
                         kStageWeight[1] * (c->bstage[1][4 + v] - c->bstage[1][v]) +
                         kStageWeight[2] * (c->bstage[2][4 + v] - c->bstage[2][v]);
            c->bflux[v] += dt * net;
        }
        c->t = c->last ? c->t_end : c->t + dt;
        c->steps += 1;
        if (dt < c->dt_min) c->dt_min = dt;
        if (dt > c->dt_max) c->dt_max = dt;
        c->troubled += (long long)c->tcount[0] + c->tcount[1] + c->tcount[2];
        c->active = 0;
    }
    if (finalize_only || c->done) return;
    // a positivity violation is reported but does not stop the run; a
    // non-finite value does
    if (c->status == -4 || !(c->t < c->t_end) || c->steps >= c->max_steps) {
        c->done = 1;
        return;
    }
    const double alpha = __longlong_as_double((long long)c->alpha_bits);
    double dt = c->cfl_num / alpha;
    // a non-finite step, or one too small to advance t, ends the run
    if (!(dt > 0.0) || !isfinite(dt) || !(c->t + dt > c->t)) {
        if (c->status == 0) {
            c->status = -4;
            c->first_bad = -1;
        }
        c->done = 1;
        return;
    }
    int last = 0;
    if (c->t + dt >= c->t_end) {
        dt = c->t_end - c->t;
        last = 1;
    }
    c->dt = dt;
    c->last = last;
    c->active = 1;
    c->alpha_bits = 0;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        c->tcount[s] = 0;
        c->eta_line[s].v = 0;
#pragma unroll
        for (int v = 0; v < 8; ++v) c->bstage[s][v] = 0.0;
    }
}

// 1D stage kernels use small tiles below this many cells (one wavefront; two
// for the hybrid stage).
constexpr int64_t kSmallTileCells = 252 * 1024;

// The fields of Ctrl that the step control works on, without the control
// block's padding: a copy this size stays in registers.
struct CtrlRegs {
    double t, dt, t_end, dt_min, dt_max, cfl_num;
    unsigned long long alpha_bits;
    unsigned int tcount[3];
    struct {
        unsigned long long v;
    } eta_line[3];
    int active;
    long long steps, max_steps, troubled;
    int last, done, status, reject;
    long long first_bad;
    double bflux[4];
    double bstage[3][8];
    long long restarts;
    int retries;
};

// COHERENT: the fields other workgroups of the running launch may have
// changed (atomics, atomic stores) are read at the point of coherence.
template <bool COHERENT>
__device__ inline CtrlRegs load_ctrl_regs(const Ctrl* c)
{
    auto ld = [](const auto* p) {
        using T = typename std::remove_cv<typename std::remove_pointer<decltype(p)>::type>::type;
        if constexpr (COHERENT)
            return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else
            return *p;
    };
    CtrlRegs r;
    r.t = c->t;
    r.dt = c->dt;
    r.t_end = c->t_end;
    r.dt_min = c->dt_min;
    r.dt_max = c->dt_max;
    r.cfl_num = c->cfl_num;
    r.alpha_bits = ld(&c->alpha_bits);
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        r.tcount[s] = ld(&c->tcount[s]);
        r.eta_line[s].v = c->eta_line[s].v;
#pragma unroll
        for (int v = 0; v < 8; ++v)
            r.bstage[s][v] = __longlong_as_double(ld(reinterpret_cast<const long long*>(&c->bstage[s][v])));
    }
    r.active = c->active;
    r.steps = c->steps;
    r.max_steps = c->max_steps;
    r.troubled = c->troubled;
    r.last = c->last;
    r.done = c->done;
    r.status = ld(&c->status);
    r.reject = ld(&c->reject);
    r.first_bad = ld(&c->first_bad);
#pragma unroll
    for (int v = 0; v < 4; ++v) r.bflux[v] = c->bflux[v];
    r.restarts = c->restarts;
    r.retries = c->retries;
    return r;
}

__device__ inline void store_ctrl_regs(Ctrl* c, const CtrlRegs& r)
{
    c->t = r.t;
    c->dt = r.dt;
    c->dt_min = r.dt_min;
    c->dt_max = r.dt_max;
    c->alpha_bits = r.alpha_bits;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        c->tcount[s] = r.tcount[s];
        c->eta_line[s].v = r.eta_line[s].v;
#pragma unroll
        for (int v = 0; v < 8; ++v) c->bstage[s][v] = r.bstage[s][v];
    }
    c->active = r.active;
    c->steps = r.steps;
    c->troubled = r.troubled;
    c->last = r.last;
    c->done = r.done;
    c->status = r.status;
    c->reject = r.reject;
    c->first_bad = r.first_bad;
#pragma unroll
    for (int v = 0; v < 4; ++v) c->bflux[v] = r.bflux[v];
    c->restarts = r.restarts;
    c->retries = r.retries;
}

// The step control run inside a stage kernel, by the workgroup that
// finishes last (1D dg_run without the positivity limiter): every other
// workgroup's atomics into the control block completed before it counted
// itself in, and the fields those atomics change are re-read here at the
// point of coherence; the rest was written before the launch.
__device__ inline void step_ctrl_in_kernel(Ctrl* c)
{
    CtrlRegs r = load_ctrl_regs<true>(c);
    step_ctrl_body(&r, 0);
    store_ctrl_regs(c, r);
    __hip_atomic_store(&c->arrive.v, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// step control (dg_util.hip)
hipError_t launch_step_ctrl(Ctrl* c, int finalize_only, hipStream_t st);
hipError_t launch_restore(const Ctrl* c, const void* src, void* dst, size_t bytes, hipStream_t st);
template <typename TB>
hipError_t launch_convert(int to_internal, int nv, int nmodes, int64_t ncell, const double* fp64,
                          StateView<TB> v, hipStream_t st);
// Conservation ledger: out[v] = cell volume x sum of the cell averages of
// variable v; part holds nv x kLedgerParts doubles of partial sums.
constexpr int kLedgerParts = 256;
template <typename TB>
hipError_t launch_ledger(int nv, int64_t ncell, StateView<TB> u, double cell_volume, double* out,
                         double* part, hipStream_t st);
template <typename TB>
hipError_t launch_check1d(int eq, int k, StateView<TB> u, int64_t n, PhysParams phys, Ctrl* c,
                          double* minvals, int pp, hipStream_t st);

}  // namespace dg
