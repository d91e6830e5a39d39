// dg_api.hip — host side of the C ABI declared in include/dg.h.
//
// The handle keeps parameters, the workspace carve-up and one instantiated
// HIP graph of G fused time steps.  dg_run replays that graph on a private
// non-blocking stream (capture is not possible on the null stream) until
// the device control block reports that t_end or the step limit was reached;
// time steps are chosen on the device, so the host only reads the control
// block between batches of replays.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <new>

#include "../../include/dg.h"
#include "dg_kernels.h"

using namespace dg;

struct dg_solver {
    dg_mesh mesh;
    dg_options opt;
    int k, eq, dim, nv, nmodes, lmax;  // nmodes: modes stored per variable
    int pk;                            // 2D P^k space in compact planes
    int64_t ncell, n_pad;
    double h[2], inv_h[2];
    size_t state_bytes, ws_bytes;
    size_t off_w, off_E, off_eta, off_tcell, off_tdata, off_aux, off_pcell;
    size_t off_corner, off_ppfail;  // 2D hybrid runs: corner values, screen verdicts
    size_t off_dv, dv_slot;  // deferred hybrid blend: 4 slots of eta[n] + E[k][n]
    void* u[3];
    unsigned char* ws;
    bool bound;
    hipStream_t user_st;
    hipStream_t run_st;
    hipGraphExec_t graph;
};

namespace {

constexpr size_t kCtrlBytes = 4096;
// aux scratch: [0..3] ledger, [4..5] minima, [8..10] per-call counters,
// [16..) a second control block, [256] and [272] the eta maxima of the
// deferred-blend slots 2 and 3 (128-byte lines of their own); from byte 4096
// the ledger's partial sums.
constexpr size_t kAuxDeferredM = 256;  // in doubles
constexpr size_t kAuxLedgerOff = 512;  // in doubles
constexpr size_t kAuxBytes = 4096 + 4 * kLedgerParts * sizeof(double);
static_assert(16 * sizeof(double) + sizeof(Ctrl) <= kAuxDeferredM * sizeof(double),
              "the second control block overlaps the deferred-blend maxima");
constexpr int kGraphSteps = 16;  // even: the three state buffers rotate with period 2

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

#define DG_HIP(call)                                   \
    do {                                               \
        hipError_t e_ = (call);                        \
        if (e_ != hipSuccess) return DG_ERR_DEVICE;    \
    } while (0)

template <typename TB>
StateView<TB> view_of(const dg_solver* s, void* base)
{
    StateView<TB> v;
    if (s->opt.precision == DG_PREC_FP64) {
        double* b = static_cast<double*>(base);
        v.m0 = b;
        v.s0 = (int64_t)s->nmodes * s->ncell;
        v.hi = reinterpret_cast<TB*>(b + s->ncell);
        v.sv = (int64_t)s->nmodes * s->ncell;
        v.sl = s->ncell;
    } else {
        double* b = static_cast<double*>(base);
        v.m0 = b;
        v.s0 = s->n_pad;
        v.hi = reinterpret_cast<TB*>(b + (size_t)s->nv * s->n_pad);
        v.sv = (int64_t)(s->nmodes - 1) * s->n_pad;
        v.sl = s->n_pad;
    }
    return v;
}

Ctrl* ctrl_of(const dg_solver* s) { return reinterpret_cast<Ctrl*>(s->ws); }
double* aux_of(const dg_solver* s) { return reinterpret_cast<double*>(s->ws + s->off_aux); }

template <typename TB>
Args1D<TB> base_args(const dg_solver* s)
{
    Args1D<TB> a;
    memset(&a, 0, sizeof a);
    a.n = s->ncell;
    a.inv_h = s->inv_h[0];
    a.periodic = s->mesh.bc[0] == DG_BC_PERIODIC;
    a.bc_lo = s->mesh.bc[0];
    a.bc_hi = s->mesh.bc[1];
    for (int v = 0; v < 4; ++v) {
        a.dir_lo[v] = s->mesh.dirichlet[0][v];
        a.dir_hi[v] = s->mesh.dirichlet[1][v];
    }
    a.phys.gamma = s->opt.gamma;
    a.phys.flux = s->opt.flux;
    a.phys.a[0] = s->opt.adv_speed[0];
    a.phys.a[1] = s->opt.adv_speed[1];
    a.check = s->eq == DG_EQ_EULER;
    a.ctrl = ctrl_of(s);
    a.pp = s->opt.positivity;
    a.reject = &ctrl_of(s)->reject;
    a.tcap = s->ncell;
    return a;
}

template <typename TB>
PPArgs pp_args(const dg_solver* s)
{
    PPArgs p;
    p.on = s->opt.positivity;
    p.phys = base_args<TB>(s).phys;
    p.reject = &ctrl_of(s)->reject;
    return p;
}

template <typename TB>
Args2D<TB> base_args2d(const dg_solver* s)
{
    Args2D<TB> a;
    memset(&a, 0, sizeof a);
    a.nx = s->mesh.n[0];
    a.ny = s->mesh.n[1];
    a.hx = s->h[0];
    a.hy = s->h[1];
    a.inv_hx = s->inv_h[0];
    a.inv_hy = s->inv_h[1];
    a.xlo = s->mesh.lo[0];
    a.ylo = s->mesh.lo[1];
    for (int i = 0; i < 4; ++i) {
        a.bc[i] = s->mesh.bc[i];
        for (int v = 0; v < 4; ++v) a.dir[i][v] = s->mesh.dirichlet[i][v];
        a.post[i] = s->mesh.post[i];
        a.pre[i] = s->mesh.pre[i];
    }
    a.shock_x0 = s->mesh.shock_x0;
    a.shock_speed = s->mesh.shock_speed;
    a.phys.gamma = s->opt.gamma;
    a.phys.flux = s->opt.flux;
    a.phys.a[0] = s->opt.adv_speed[0];
    a.phys.a[1] = s->opt.adv_speed[1];
    // with the positivity limiter, point values sit at its margin: the
    // stage kernel's point check is off and only averages are checked
    a.check = s->eq == DG_EQ_EULER && !s->opt.positivity;
    a.ctrl = ctrl_of(s);
    a.tcap = s->ncell;
    a.pk = s->pk;
    if (s->opt.positivity) {
        a.pp = 1;
        a.pcount = &ctrl_of(s)->pcount.v;
        a.pcell = reinterpret_cast<long long*>(s->ws + s->off_pcell);
        a.pcap = s->ncell;
        a.reject = &ctrl_of(s)->reject;
    }
    // mesh factors of (c_fx, c_fy): (hx, hy) printed in Sec. 2.4, (hy, hx)
    // printed in Sec. 3.2, or none
    const int rd = s->opt.cf_reading;
    a.cfmx = rd == 0 ? a.hx : rd == 1 ? a.hy : 1.0;
    a.cfmy = rd == 0 ? a.hy : rd == 1 ? a.hx : 1.0;
    // jump weights of the multi-index (a1, a2), m = a1 + a2: hx (m = 0),
    // m(m+1) hx^(m+1) (2/hx)^a1 (2/hy)^a2 (x edges); likewise with hy
    for (int a1 = 0; a1 < 4; ++a1)
        for (int a2 = 0; a2 < 4; ++a2) {
            const int m = a1 + a2;
            const double d = pow(2.0 / a.hx, a1) * pow(2.0 / a.hy, a2);
            a.jsx[a1 * 4 + a2] = m == 0 ? a.hx : m * (m + 1.0) * pow(a.hx, m + 1) * d;
            a.jsy[a1 * 4 + a2] = m == 0 ? a.hy : m * (m + 1.0) * pow(a.hy, m + 1) * d;
        }
    return a;
}

template <typename TB>
int stage_impl(dg_solver* s, int stage, double dt)
{
    if (s->dim == 2) {
        Args2D<TB> a = base_args2d<TB>(s);
        a.un = view_of<TB>(s, s->u[0]);
        a.us = view_of<TB>(s, s->u[stage]);
        a.out = view_of<TB>(s, s->ws + s->off_w);
        a.stage = stage;
        a.dt_host = dt;
        a.t_host = 0.0;
        DG_HIP(launch_stage2d<TB>(s->eq, s->k, a, s->user_st));
        return DG_OK;
    }
    Args1D<TB> a = base_args<TB>(s);
    a.un = view_of<TB>(s, s->u[0]);
    a.us = view_of<TB>(s, s->u[stage]);
    a.out = view_of<TB>(s, s->ws + s->off_w);
    a.stage = stage;
    a.dt_host = dt;
    a.pp = 0;  // the limiter belongs to the post-stage operator
    DG_HIP(launch_stage1d<TB>(s->eq, s->k, a, 0, s->user_st));
    return DG_OK;
}

template <typename TB>
int filter_impl(dg_solver* s, int stage, double dt)
{
    void* target = stage == 0 ? s->u[1] : stage == 1 ? s->u[2] : s->u[0];
    if (s->opt.filter == DG_FILTER_NONE) {
        DG_HIP(hipMemcpyAsync(target, s->ws + s->off_w, s->state_bytes, hipMemcpyDeviceToDevice,
                              s->user_st));
        if (s->opt.positivity) {
            const StateView<TB> t = view_of<TB>(s, target);
            if (s->dim == 2)
                DG_HIP(launch_pp2d<TB>(s->k, t, s->ncell, nullptr, nullptr, s->ncell, ctrl_of(s), 0,
                                       s->pk, pp_args<TB>(s), s->user_st));
            else
                DG_HIP(launch_blend_all1d<TB>(s->nv, s->k, t, t, s->ncell, nullptr, nullptr, nullptr,
                                              nullptr, pp_args<TB>(s), s->user_st));
        }
        return DG_OK;
    }
    if (s->dim == 2) {
        Args2D<TB> a = base_args2d<TB>(s);
        a.stage = stage;
        a.dt_host = dt;
        a.t_host = 0.0;
        a.E_out = reinterpret_cast<double*>(s->ws + s->off_E);
        if (a.pp) DG_HIP(hipMemsetAsync(a.pcount, 0, sizeof *a.pcount, s->user_st));
        if (s->opt.filter == DG_FILTER_JUMP) {
            a.us = view_of<TB>(s, s->ws + s->off_w);
            a.out = view_of<TB>(s, target);
            DG_HIP(launch_filter2d<TB>(s->eq, s->k, a, s->user_st));
            if (a.pp)
                DG_HIP(launch_pp2d<TB>(s->k, a.out, s->ncell, a.pcount, a.pcell, a.pcap, ctrl_of(s), 0,
                                       s->pk, pp_args<TB>(s), s->user_st));
            return DG_OK;
        }
        // hybrid: the unfiltered output goes to the target, pass A records
        // the troubled cells, pass B blends them in place
        DG_HIP(hipMemcpyAsync(target, s->ws + s->off_w, s->state_bytes, hipMemcpyDeviceToDevice,
                              s->user_st));
        double* aux = aux_of(s);
        unsigned long long* eta_bits = reinterpret_cast<unsigned long long*>(aux + 8);
        unsigned int* tcount = reinterpret_cast<unsigned int*>(aux + 9);
        DG_HIP(hipMemsetAsync(aux + 8, 0, 2 * sizeof(double), s->user_st));
        a.us = view_of<TB>(s, target);
        a.out = a.us;
        a.eta_acc = eta_bits;
        a.tcount = tcount;
        a.tcell = reinterpret_cast<long long*>(s->ws + s->off_tcell);
        a.tdata = reinterpret_cast<double*>(s->ws + s->off_tdata);
        a.eta_out = reinterpret_cast<double*>(s->ws + s->off_eta);
        DG_HIP(launch_indicator2d<TB>(s->eq, s->k, a, s->user_st));
        DG_HIP(launch_troubled2d<TB>(s->eq, s->k, a, s->user_st));
        DG_HIP(launch_blend2d<TB>(s->nv, s->k, a, pp_args<TB>(s), s->user_st));
        if (a.pp)
            DG_HIP(launch_pp2d<TB>(s->k, a.out, s->ncell, a.pcount, a.pcell, a.pcap, ctrl_of(s), 0,
                                   s->pk, pp_args<TB>(s), s->user_st));
        return DG_OK;
    }
    Args1D<TB> a = base_args<TB>(s);
    a.us = view_of<TB>(s, s->ws + s->off_w);
    a.out = view_of<TB>(s, target);
    a.stage = stage;
    a.dt_host = dt;
    a.E_out = reinterpret_cast<double*>(s->ws + s->off_E);
    if (s->opt.filter == DG_FILTER_JUMP) {
        DG_HIP(launch_filter1d<TB>(s->eq, s->k, a, 1, s->user_st));
        return DG_OK;
    }
    double* aux = aux_of(s);
    unsigned long long* eta_bits = reinterpret_cast<unsigned long long*>(aux + 8);
    unsigned int* tcount = reinterpret_cast<unsigned int*>(aux + 9);
    DG_HIP(hipMemsetAsync(aux + 8, 0, 2 * sizeof(double), s->user_st));
    a.eta_out = reinterpret_cast<double*>(s->ws + s->off_eta);
    a.eta_acc = eta_bits;
    DG_HIP(launch_filter1d<TB>(s->eq, s->k, a, 2, s->user_st));
    DG_HIP(launch_blend_all1d<TB>(s->nv, s->k, a.us, a.out, s->ncell, a.E_out, a.eta_out, eta_bits,
                                  tcount, pp_args<TB>(s), s->user_st));
    return DG_OK;
}

template <typename TB>
int maxwave_impl(dg_solver* s, unsigned long long* acc, hipStream_t st)
{
    if (s->dim == 2) {
        DG_HIP(launch_maxwave2d<TB>(s->eq, view_of<TB>(s, s->u[0]), s->mesh.n[0], s->mesh.n[1],
                                    s->inv_h[0], s->inv_h[1], base_args2d<TB>(s).phys, acc,
                                    ctrl_of(s), st));
        return DG_OK;
    }
    DG_HIP(launch_maxwave1d<TB>(s->eq, view_of<TB>(s, s->u[0]), s->ncell,
                                base_args<TB>(s).phys, acc, ctrl_of(s), st));
    return DG_OK;
}

// Record G fused steps (rotation A->B, (B,A)->C, (C,A)->B; then the mirror)
// on the capture stream.
// 1D hybrid without the positivity limiter: pass B is not a kernel of its
// own; pass A records eta and the exponents per cell, and every stage that
// loads a state owing its blend applies it on load (blend_apply).  Slots
// 0 and 1 hold stages 0 and 1 of a step, slots 2 and 3 stage 2 of even and
// odd steps (u^n of the next step still owes that blend).
bool deferred_blend_on(const dg_solver* s) { return s->dv_slot != 0; }

template <typename TB>
typename Args1D<TB>::Deferred dv_view(const dg_solver* s, int slot)
{
    typename Args1D<TB>::Deferred d;
    TB* base = reinterpret_cast<TB*>(s->ws + s->off_dv + (size_t)slot * s->dv_slot);
    d.eta = base;
    d.E = base + s->ncell;
    double* aux = reinterpret_cast<double*>(s->ws + s->off_aux);
    Ctrl* c = reinterpret_cast<Ctrl*>(s->ws);
    d.M = slot < 2 ? &c->eta_line[slot].v
                   : reinterpret_cast<const unsigned long long*>(aux + kAuxDeferredM + 16 * (slot - 2));
    return d;
}

// 1D jump filter or no filter: the three stages of a step run in one launch
// on tiles with a 6-cell (3-cell) halo, reading u^n once and writing u^{n+1}
// once.  (The hybrid needs a global max per stage.)  With the positivity
// limiter a stage that leaves an inadmissible average flags the step, whose
// output is then replaced by u^n and retried, as with per-stage launches.
bool fused_step(const dg_solver* s)
{
    return s->dim == 1 && s->opt.filter != DG_FILTER_HYBRID;
}

// 1D hybrid runs with the deferred blend on small grids (small tiles, where
// launches and their latency bound the step): the step control runs at the
// end of each step's last stage, in the workgroup that finishes last,
// instead of as a kernel of its own before the next step (the run's first
// step is scheduled before the first batch of steps).
bool folded_ctrl(const dg_solver* s)
{
    return s->dim == 1 && deferred_blend_on(s) && s->ncell < kSmallTileCells;
}

// 2D hybrid: the stage kernel writes its output's corner values (and the
// limiter screen's verdicts) for the indicator that follows it
template <typename TB>
void corner_args(const dg_solver* s, Args2D<TB>& a)
{
    a.corner = reinterpret_cast<TB*>(s->ws + s->off_corner);
    a.cstride = s->ncell;
    a.ppfail = s->opt.positivity ? reinterpret_cast<unsigned char*>(s->ws + s->off_ppfail) : nullptr;
}

template <typename TB>
int record_steps(dg_solver* s, int G, hipStream_t st)
{
    Ctrl* c = ctrl_of(s);
    const int fmode = s->opt.filter == DG_FILTER_NONE ? 0 : s->opt.filter == DG_FILTER_JUMP ? 1 : 2;
    long long* tcell = reinterpret_cast<long long*>(s->ws + s->off_tcell);
    double* tdata = reinterpret_cast<double*>(s->ws + s->off_tdata);
    for (int i = 0; i < G; ++i) {
        void* A = (i % 2 == 0) ? s->u[0] : s->u[1];
        void* B = (i % 2 == 0) ? s->u[1] : s->u[0];
        void* Cb = s->u[2];
        if (!folded_ctrl(s)) DG_HIP(launch_step_ctrl(c, 0, st));
        if (s->dim == 2) {
            for (int stage = 0; stage < 3; ++stage) {
                void* target = stage == 1 ? Cb : B;
                void* src = stage == 0 ? A : stage == 1 ? B : Cb;
                Args2D<TB> a = base_args2d<TB>(s);
                a.un = view_of<TB>(s, A);
                a.us = view_of<TB>(s, src);
                a.stage = stage;
                a.dt_from_ctrl = 1;
                a.alpha_acc = stage == 2 ? &c->alpha_bits : nullptr;
                Args2D<TB> f = base_args2d<TB>(s);
                f.stage = stage;
                f.dt_from_ctrl = 1;
                if (fmode == 1) {
                    // residual -> workspace, filter workspace -> target
                    a.out = view_of<TB>(s, s->ws + s->off_w);
                    DG_HIP(launch_stage2d<TB>(s->eq, s->k, a, st));
                    f.us = a.out;
                    f.out = view_of<TB>(s, target);
                    DG_HIP(launch_filter2d<TB>(s->eq, s->k, f, st));
                } else {
                    a.out = view_of<TB>(s, target);
                    if (fmode == 2) {
                        corner_args<TB>(s, a);
                        corner_args<TB>(s, f);
                    }
                    DG_HIP(launch_stage2d<TB>(s->eq, s->k, a, st));
                    if (fmode == 2) {
                        // hybrid: pass A (indicator, troubled list), pass B
                        // (exponents, blend and limiter of the troubled cells)
                        f.us = f.out = a.out;
                        f.eta_acc = &c->eta_line[stage].v;
                        f.tcount = &c->tcount[stage];
                        f.tcell = tcell;
                        f.tdata = tdata;
                        DG_HIP(launch_indicator2d<TB>(s->eq, s->k, f, st));
                        DG_HIP(launch_troubled2d<TB>(s->eq, s->k, f, st));
                        DG_HIP(launch_blend2d<TB>(s->nv, s->k, f, pp_args<TB>(s), st));
                    }
                }
                // positivity limiter on the cells the post-stage kernels
                // listed (without a filter: on every cell)
                if (s->opt.positivity)
                    DG_HIP(launch_pp2d<TB>(s->k, view_of<TB>(s, target), s->ncell,
                                           fmode ? f.pcount : nullptr, f.pcell, f.pcap, c, 1, s->pk,
                                           pp_args<TB>(s), st));
            }
            // a rejected step is undone (u^n copied over its output) and
            // retried with half dt by the next step control
            if (s->opt.positivity) DG_HIP(launch_restore(c, A, B, s->state_bytes, st));
            continue;
        }
        if (fused_step(s)) {
            // the whole step in one launch: u^n (A) -> u^{n+1} (B)
            Args1D<TB> a = base_args<TB>(s);
            a.un = a.us = view_of<TB>(s, A);
            a.out = view_of<TB>(s, B);
            a.stage = 2;
            a.dt_from_ctrl = 1;
            a.bflux = &c->bstage[0][0];
            a.alpha_acc = &c->alpha_bits;
            DG_HIP(launch_stage1d<TB>(s->eq, s->k, a, fmode, st, 3));
            if (s->opt.positivity) DG_HIP(launch_restore(c, A, B, s->state_bytes, st));
            continue;
        }
        const bool dfr = deferred_blend_on(s);
        const int prev2 = 2 + ((i + 1) & 1), cur2 = 2 + (i & 1);
        for (int stage = 0; stage < 3; ++stage) {
            Args1D<TB> a = base_args<TB>(s);
            a.un = view_of<TB>(s, A);
            a.us = view_of<TB>(s, stage == 0 ? A : stage == 1 ? B : Cb);
            a.out = view_of<TB>(s, stage == 1 ? Cb : B);
            a.stage = stage;
            a.dt_from_ctrl = 1;
            a.bflux = &c->bstage[stage][0];
            a.alpha_acc = stage == 2 ? &c->alpha_bits : nullptr;
            a.eta_acc = &c->eta_line[stage].v;
            a.tcount = &c->tcount[stage];
            a.tcell = tcell;
            a.tdata = tdata;
            if (dfr) {
                // u^n owes the blend of the previous step's last stage; u^(s)
                // (s >= 1) the blend of stage s - 1 of this step
                const auto dv_out = dv_view<TB>(s, stage < 2 ? stage : cur2);
                a.dv_eta = const_cast<TB*>(dv_out.eta);
                a.dv_E = const_cast<TB*>(dv_out.E);
                a.bl_un = dv_view<TB>(s, prev2);
                a.bl_us = stage == 0 ? a.bl_un : dv_view<TB>(s, stage - 1);
                if (stage == 2) a.eta_acc = const_cast<unsigned long long*>(dv_out.M);
                a.fold_ctrl = stage == 2 && folded_ctrl(s);
                // this step's last-stage maximum is cleared before stage 2
                if (stage == 1) a.zero_bits = const_cast<unsigned long long*>(dv_view<TB>(s, cur2).M);
            }
            DG_HIP(launch_stage1d<TB>(s->eq, s->k, a, fmode, st));
            if (dfr) continue;
            if (fmode == 2)
                DG_HIP(launch_blend1d<TB>(s->nv, s->k, a.out, &c->tcount[stage], tcell, tdata,
                                          &c->eta_line[stage].v, c, 1, s->ncell,
                                          pp_args<TB>(s), st));
        }
        // positivity limiter: a rejected step is undone (u^n copied over its
        // output) and retried with half dt by the next step control
        if (s->opt.positivity) DG_HIP(launch_restore(c, A, B, s->state_bytes, st));
    }
    return DG_OK;
}

template <typename TB>
int build_graph(dg_solver* s)
{
    if (s->graph) {
        (void)hipGraphExecDestroy(s->graph);
        s->graph = nullptr;
    }
    hipGraph_t g = nullptr;
    DG_HIP(hipStreamBeginCapture(s->run_st, hipStreamCaptureModeThreadLocal));
    int rc = record_steps<TB>(s, kGraphSteps, s->run_st);
    hipError_t e = hipStreamEndCapture(s->run_st, &g);
    if (rc != DG_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return DG_ERR_DEVICE;
    e = hipGraphInstantiate(&s->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        s->graph = nullptr;
        return DG_ERR_DEVICE;
    }
    return DG_OK;
}

template <typename TB>
int report_impl(dg_solver* s, dg_report* rep)
{
    hipStream_t st = s->run_st;
    double* aux = aux_of(s);
    // aux[0..3] ledger, aux[4..5] min rho / min p (as ordered bits)
    unsigned long long inf_bits = (unsigned long long)0x7ff0000000000000ULL;
    unsigned long long init[2] = {inf_bits, inf_bits};
    DG_HIP(hipStreamSynchronize(st));
    DG_HIP(hipMemcpy(aux + 4, init, sizeof init, hipMemcpyHostToDevice));
    const double vol = s->dim == 1 ? s->h[0] : s->h[0] * s->h[1];
    DG_HIP(launch_ledger<TB>(s->nv, s->ncell, view_of<TB>(s, s->u[0]), vol, aux, aux + kAuxLedgerOff,
                             st));
    if (s->dim == 1)
        DG_HIP(launch_check1d<TB>(s->eq, s->k, view_of<TB>(s, s->u[0]), s->ncell,
                                  base_args<TB>(s).phys, ctrl_of(s), aux + 4, s->opt.positivity, st));
    Ctrl c;
    double hv[6];
    DG_HIP(hipMemcpyAsync(&c, ctrl_of(s), sizeof c, hipMemcpyDeviceToHost, st));
    DG_HIP(hipMemcpyAsync(hv, aux, sizeof hv, hipMemcpyDeviceToHost, st));
    DG_HIP(hipStreamSynchronize(st));
    if (rep) {
        memset(rep, 0, sizeof *rep);
        rep->t = c.t;
        rep->dt_min = c.dt_min;
        rep->dt_max = c.dt_max;
        for (int v = 0; v < 4; ++v) {
            rep->ledger[v] = v < s->nv ? hv[v] : 0.0;
            rep->boundary_flux[v] = c.bflux[v];
        }
        rep->troubled_cells = c.troubled;
        rep->min_rho = s->eq == DG_EQ_EULER ? hv[4] : NAN;
        rep->min_p = s->eq == DG_EQ_EULER ? hv[5] : NAN;
        rep->max_exponent = NAN;
        rep->status = c.status;
        rep->first_bad_cell = c.status ? c.first_bad : -1;
        rep->steps = c.steps;
        rep->restarts = c.restarts;
    }
    return c.status;
}

template <typename TB>
int run_impl(dg_solver* s, double t_end, int64_t max_steps, dg_report* rep)
{
    DG_HIP(hipStreamSynchronize(s->user_st));
    hipStream_t st = s->run_st;
    Ctrl c;
    DG_HIP(hipMemcpy(&c, ctrl_of(s), sizeof c, hipMemcpyDeviceToHost));
    const long long steps0 = c.steps;
    c.t_end = t_end;
    c.max_steps = steps0 + max_steps;
    c.done = 0;
    c.active = 0;
    c.reject = 0;
    c.retries = 0;
    c.dt_min = INFINITY;
    c.dt_max = 0.0;
    c.alpha_bits = 0;
    c.arrive.v = 0;
    c.cfl_num = s->dim == 1 ? s->opt.cfl * s->h[0] : s->opt.cfl;
    DG_HIP(hipMemcpy(ctrl_of(s), &c, sizeof c, hipMemcpyHostToDevice));
    // Small-grid hybrid runs with the folded step control launch their steps
    // directly on the stream: replayed from a graph, the same kernels ran
    // slower on the device (35.5 against 32.4 us per step, where the host's
    // launch rate was then the limit).  Every other run replays a graph.
    const bool direct = folded_ctrl(s);
    if (!direct && !s->graph) {
        int rc = build_graph<TB>(s);
        if (rc) return rc;
    }
    int rc = maxwave_impl<TB>(s, &ctrl_of(s)->alpha_bits, st);
    if (rc) return rc;
    // deferred hybrid blend: the run's first step owes no blend on u^n
    if (deferred_blend_on(s))
        DG_HIP(hipMemsetAsync(s->ws + s->off_dv + 3 * s->dv_slot, 0, s->ncell * sizeof(TB), st));
    // folded step control: the first step is scheduled here, every later one
    // at the end of the step before it
    const bool folded = folded_ctrl(s);
    if (folded) DG_HIP(launch_step_ctrl(ctrl_of(s), 0, st));
    // Replays: batches double in size between control reads, never beyond
    // the replays the remaining step budget needs; a remainder of fewer than
    // kGraphSteps steps is launched directly, rounded up to an even count
    // (every launch sequence then keeps the buffer roles' period of 2; a
    // slot past the budget finds the run done and exits at once).  With the
    // positivity limiter a rejected step is retried, so the budget is
    // re-read.
    const long long restarts0 = c.restarts;
    long long batch = 1, completed = 0;
    for (;;) {
        const long long rem = max_steps - completed;
        if (rem <= 0) break;
        long long nb = rem / kGraphSteps;
        const int tail = (int)(rem % kGraphSteps);
        if (nb > batch) nb = batch;
        for (long long r = 0; r < nb; ++r) {
            if (!direct) {
                DG_HIP(hipGraphLaunch(s->graph, st));
                continue;
            }
            const int rs = record_steps<TB>(s, kGraphSteps, st);
            if (rs) return rs;
        }
        if (nb < batch && tail > 0) {
            const int rs = record_steps<TB>(s, tail + (tail & 1), st);
            if (rs) return rs;
        }
        Ctrl cr;
        DG_HIP(hipMemcpyAsync(&cr, ctrl_of(s), sizeof cr, hipMemcpyDeviceToHost, st));
        DG_HIP(hipStreamSynchronize(st));
        if (cr.done) break;
        // the last step of a replay has run but is finalised by the next
        // step control, unless it was rejected (with the folded control it
        // is finalised, and an active step is the next one, not yet run)
        completed = cr.steps - steps0 + ((!folded && cr.active && !cr.reject) ? 1 : 0);
        batch = batch < 64 ? batch * 2 : 64;
    }
    DG_HIP(launch_step_ctrl(ctrl_of(s), 1, st));
    DG_HIP(hipMemcpyAsync(&c, ctrl_of(s), sizeof c, hipMemcpyDeviceToHost, st));
    DG_HIP(hipStreamSynchronize(st));
    // every executed step (finalised or rejected) swaps the buffer roles
    const long long executed = c.steps - steps0 + c.restarts - restarts0;
    if (executed & 1)
        DG_HIP(hipMemcpyAsync(s->u[0], s->u[1], s->state_bytes, hipMemcpyDeviceToDevice, st));
    // deferred hybrid blend: the last step's output still owes its blend
    if (deferred_blend_on(s) && executed > 0)
        DG_HIP(launch_deferred_blend1d<TB>(s->nv, s->k, view_of<TB>(s, s->u[0]), s->ncell,
                                           dv_view<TB>(s, 2 + (int)((executed - 1) & 1)), st));
    return report_impl<TB>(s, rep);
}

bool is_fp64(const dg_solver* s) { return s->opt.precision == DG_PREC_FP64; }

// Events around each launch of the fused stage kernel (rotation slot 0 of
// dg_run: A = u_n read-only, outputs to u_a / u_b).  The hybrid list and
// the CFL accumulator point into the aux scratch, whose counters are
// cleared by a one-thread kernel before each timed launch.
// Average duration of `reps` back-to-back launches of one kernel on the run
// stream, from HIP events recorded before the first and after the last
// launch (one warm-up launch first; the scratch control block's per-step
// accumulators are cleared before the timed launches, and the troubled
// lists saturate at their capacity).
template <typename F>
int time_launches(dg_solver* s, Ctrl* scratch, int reps, F launch, double* avg_us)
{
    hipStream_t st = s->run_st;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = DG_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = DG_ERR_DEVICE;
    if (rc == DG_OK && launch_step_ctrl(scratch, 2, st) != hipSuccess) rc = DG_ERR_DEVICE;
    if (rc == DG_OK && launch() != hipSuccess) rc = DG_ERR_DEVICE;
    if (rc == DG_OK && launch_step_ctrl(scratch, 2, st) != hipSuccess) rc = DG_ERR_DEVICE;
    if (rc == DG_OK && hipEventRecord(e0, st) != hipSuccess) rc = DG_ERR_DEVICE;
    for (int r = 0; r < reps && rc == DG_OK; ++r)
        if (launch() != hipSuccess) rc = DG_ERR_DEVICE;
    if (rc == DG_OK && hipEventRecord(e1, st) != hipSuccess) rc = DG_ERR_DEVICE;
    if (rc == DG_OK && hipEventSynchronize(e1) != hipSuccess) rc = DG_ERR_DEVICE;
    float ms = 0.f;
    if (rc == DG_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = DG_ERR_DEVICE;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (rc == DG_OK) *avg_us = 1000.0 * ms / reps;
    return rc;
}

template <typename TB>
int time_impl(dg_solver* s, int stage, double dt, int reps, double* avg_us)
{
    hipStream_t st = s->run_st;
    const int fmode = s->opt.filter == DG_FILTER_NONE ? 0 : s->opt.filter == DG_FILTER_JUMP ? 1 : 2;
    double* aux = aux_of(s);
    Ctrl* scratch = reinterpret_cast<Ctrl*>(aux + 16);  // a second control block in aux
    if (s->dim == 2) {
        // which 0..2: residual kernel of that stage (u_n, u_a, u_b -> workspace);
        // which 3..5: the filter (jump: workspace -> u_a) or hybrid pass A (on u_a)
        const int which = stage;
        Args2D<TB> a = base_args2d<TB>(s);
        a.ctrl = scratch;
        a.stage = which % 3;
        a.dt_host = dt;
        a.un = view_of<TB>(s, s->u[0]);
        a.us = view_of<TB>(s, s->u[which % 3]);
        a.out = view_of<TB>(s, s->ws + s->off_w);
        a.alpha_acc = a.stage == 2 ? &scratch->alpha_bits : nullptr;
        Args2D<TB> f = base_args2d<TB>(s);
        f.ctrl = scratch;
        f.stage = which % 3;
        f.dt_host = dt;
        f.us = fmode == 1 ? view_of<TB>(s, s->ws + s->off_w) : view_of<TB>(s, s->u[1]);
        f.out = view_of<TB>(s, s->u[1]);
        f.eta_acc = &scratch->eta_line[0].v;
        f.tcount = &scratch->tcount[0];
        f.tcell = reinterpret_cast<long long*>(s->ws + s->off_tcell);
        f.tdata = reinterpret_cast<double*>(s->ws + s->off_tdata);
        if (fmode == 2) {
            // as in dg_run: the stage kernel hands the corner values over
            corner_args<TB>(s, a);
            corner_args<TB>(s, f);
        }
        auto launch = [&]() {
            return which < 3   ? launch_stage2d<TB>(s->eq, s->k, a, st)
                 : fmode == 1 ? launch_filter2d<TB>(s->eq, s->k, f, st)
                              : launch_indicator2d<TB>(s->eq, s->k, f, st);
        };
        return time_launches(s, scratch, reps, launch, avg_us);
    }
    if (stage == 6) {
        // the fused step kernel of dg_run (u_n -> u_a)
        if (!fused_step(s)) return DG_ERR_ARG;
        Args1D<TB> a = base_args<TB>(s);
        a.un = a.us = view_of<TB>(s, s->u[0]);
        a.out = view_of<TB>(s, s->u[1]);
        a.stage = 2;
        a.dt_host = dt;
        a.ctrl = scratch;
        a.reject = &scratch->reject;
        a.bflux = &scratch->bstage[0][0];
        a.alpha_acc = &scratch->alpha_bits;
        auto launch3 = [&]() { return launch_stage1d<TB>(s->eq, s->k, a, fmode, st, 3); };
        return time_launches(s, scratch, reps, launch3, avg_us);
    }
    Args1D<TB> a = base_args<TB>(s);
    a.un = view_of<TB>(s, s->u[0]);
    a.us = view_of<TB>(s, stage == 0 ? s->u[0] : stage == 1 ? s->u[1] : s->u[2]);
    a.out = view_of<TB>(s, stage == 1 ? s->u[2] : s->u[1]);
    a.stage = stage;
    a.dt_host = dt;
    a.ctrl = scratch;
    a.reject = &scratch->reject;
    a.bflux = &scratch->bstage[stage][0];
    a.alpha_acc = stage == 2 ? &scratch->alpha_bits : nullptr;
    a.eta_acc = &scratch->eta_line[stage].v;
    a.tcount = &scratch->tcount[stage];
    a.tcell = reinterpret_cast<long long*>(s->ws + s->off_tcell);
    a.tdata = reinterpret_cast<double*>(s->ws + s->off_tdata);
    if (fmode == 2 && deferred_blend_on(s)) {
        // as dg_run launches it: eta / exponents per cell out, blends owed by
        // the inputs applied on load (their slots hold the last run's values)
        const auto dv_out = dv_view<TB>(s, stage);
        a.dv_eta = const_cast<TB*>(dv_out.eta);
        a.dv_E = const_cast<TB*>(dv_out.E);
        a.bl_un = dv_view<TB>(s, 3);
        a.bl_us = stage == 0 ? a.bl_un : dv_view<TB>(s, stage - 1);
        // with the step control folded into the last stage, as dg_run has it
        // (it then works on the second control block)
        a.fold_ctrl = stage == 2 && folded_ctrl(s);
    }
    auto launch = [&]() { return launch_stage1d<TB>(s->eq, s->k, a, fmode, st); };
    return time_launches(s, scratch, reps, launch, avg_us);
}

// ---------------------------------------------------------------------------
// Allocation-free CFL reduction (dg_max_wavespeed_noalloc).  Its scratch --
// one partial maximum and one first-bad-cell entry per workgroup, and the
// result -- lives in a file-scope device array, one copy per GPU, held until
// the process ends.  Host code never uses the array's name as an address: the
// address is taken once per device with hipGetSymbolAddress and kept.
constexpr int kNoallocBlocks = 65536;          // workgroups of 256 cells
struct NoallocScratch {
    double part[kNoallocBlocks];               // per-workgroup maximum of lambda
    long long bad[kNoallocBlocks];             // per workgroup: first bad cell or -1
    int code[kNoallocBlocks];                  // per workgroup: 0, -5 or -4
    double alpha;                              // result
    long long first_bad;
    int status;
};

__device__ __align__(256) NoallocScratch scratch;

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
NoallocScratch* g_noalloc_ptr[kMaxDevices];

// Address of this device's scratch (taken once per device, with the device
// current); nullptr on failure.
NoallocScratch* noalloc_scratch()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        g_noalloc_ptr[dev] = static_cast<NoallocScratch*>(p);
    }
    return g_noalloc_ptr[dev];
}

// The wave speed of one cell average, as the CFL kernels compute it: 1D
// |f'(u)| (Euler |u| + c); 2D lambda_x / h_x + lambda_y / h_y.
template <int EQ, int DIM>
__device__ __forceinline__ double cell_lambda(const double* ub, const PhysParams& ph, double ihx,
                                              double ihy)
{
    if constexpr (DIM == 1) {
        return Phys1D<EQ>::speed(ub, ph);
    } else if constexpr (EQ == ADV) {
        return fabs(ph.a[0]) * ihx + fabs(ph.a[1]) * ihy;
    } else {
        const double ir = trcp<double>(ub[0]);
        const double vx = ub[1] * ir, vy = ub[2] * ir;
        const double pr = (ph.gamma - 1.0) * (ub[3] - 0.5 * (ub[1] * vx + ub[2] * vy));
        const double c = tsqrt<double>(ph.gamma * pr * ir);
        return (fabs(vx) + c) * ihx + (fabs(vy) + c) * ihy;
    }
}

// Pass 1: workgroup b reduces cells [256 b, 256 b + 256) into part[b], with
// the first inadmissible (-5) or non-finite (-4) cell of the workgroup.
template <int EQ, int DIM>
__global__ __launch_bounds__(256) void noalloc_part_kernel(const double* m0, int64_t s0, int64_t n,
                                                           PhysParams ph, double ihx, double ihy,
                                                           NoallocScratch* sc)
{
    constexpr int NV = EQ == EULER ? (DIM == 1 ? 3 : 4) : 1;
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double lam = 0.0;
    int code = 0;
    if (c < n) {
        double ub[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) ub[v] = m0[v * s0 + c];
        lam = cell_lambda<EQ, DIM>(ub, ph, ihx, ihy);
        if constexpr (EQ == EULER) {
            const double p = DIM == 1 ? (ph.gamma - 1.0) * (ub[2] - 0.5 * ub[1] * ub[1] / ub[0])
                                      : (ph.gamma - 1.0) * (ub[NV - 1] - 0.5 * (ub[1] * ub[1] + ub[2] * ub[2]) / ub[0]);
            if (!(ub[0] > 0.0) || !(p > 0.0)) code = (isfinite(ub[0]) && isfinite(p)) ? -5 : -4;
        }
        if (!isfinite(lam)) code = -4;
    }
    __shared__ double smax[4];
    __shared__ long long sbad[4];
    __shared__ int scode[4];
    const double z = wave_max(lam);
    // first bad cell of the wavefront (lowest lane with a code)
    const unsigned long long mask = __ballot(code != 0);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    long long bad = -1;
    int bcode = 0;
    if (mask) {
        const int first = __ffsll((long long)mask) - 1;
        bad = (int64_t)blockIdx.x * 256 + w * 64 + first;
        bcode = __shfl(code, first, 64);
    }
    if (lane == 0) {
        smax[w] = z;
        sbad[w] = bad;
        scode[w] = bcode;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = smax[0];
        long long b = -1;
        int cd = 0;
        for (int i = 0; i < 4; ++i) {
            m = (smax[i] > m || smax[i] != smax[i]) ? smax[i] : m;
            if (b < 0 && sbad[i] >= 0) {
                b = sbad[i];
                cd = scode[i];
            }
        }
        sc->part[blockIdx.x] = m;
        sc->bad[blockIdx.x] = b;
        sc->code[blockIdx.x] = cd;
    }
}

// Pass 2: one workgroup reduces the nb partial maxima in a fixed order.
__global__ __launch_bounds__(256) void noalloc_final_kernel(int nb, NoallocScratch* sc)
{
    __shared__ double smax[256];
    __shared__ long long sbad[256];
    __shared__ int scode[256];
    double m = 0.0;
    long long b = -1;
    int cd = 0;
    for (int i = threadIdx.x; i < nb; i += 256) {
        const double v = sc->part[i];
        m = (v > m || v != v) ? v : m;
        if (b < 0 && sc->bad[i] >= 0) {
            b = sc->bad[i];
            cd = sc->code[i];
        }
    }
    smax[threadIdx.x] = m;
    sbad[threadIdx.x] = b;
    scode[threadIdx.x] = cd;
    __syncthreads();
    if (threadIdx.x == 0) {
        // the first bad cell is the smallest index over the threads
        double mm = smax[0];
        long long bb = -1;
        int cc = 0;
        for (int i = 0; i < 256; ++i) {
            mm = (smax[i] > mm || smax[i] != smax[i]) ? smax[i] : mm;
            if (sbad[i] >= 0 && (bb < 0 || sbad[i] < bb)) {
                bb = sbad[i];
                cc = scode[i];
            }
        }
        sc->alpha = mm;
        sc->first_bad = bb;
        sc->status = cc;
    }
}

template <int EQ, int DIM>
hipError_t launch_noalloc(const double* m0, int64_t s0, int64_t n, PhysParams ph, double ihx,
                          double ihy, NoallocScratch* sc, hipStream_t st)
{
    const int nb = (int)((n + 255) / 256);
    hipLaunchKernelGGL((noalloc_part_kernel<EQ, DIM>), dim3(nb), dim3(256), 0, st, m0, s0, n, ph, ihx,
                       ihy, sc);
    hipLaunchKernelGGL(noalloc_final_kernel, dim3(1), dim3(256), 0, st, nb, sc);
    return hipGetLastError();
}

}  // namespace

extern "C" {

const char* dg_strerror(int code)
{
    switch (code) {
    case DG_OK: return "ok";
    case DG_ERR_ARG: return "invalid argument";
    case DG_ERR_UNSUPPORTED: return "unsupported degree/dimension/equation";
    case DG_ERR_DEVICE: return "HIP runtime error";
    case DG_ERR_NONFINITE: return "non-finite value in state or time step";
    case DG_ERR_POSITIVITY: return "non-positive density or pressure";
    case DG_ERR_STATE: return "buffers not bound or call out of order";
    default: return "unknown error";
    }
}

int dg_create(const dg_mesh* mesh, int degree, int equation, const dg_options* opt, dg_solver** out)
{
    if (!mesh || !opt || !out) return DG_ERR_ARG;
    *out = nullptr;
    if (mesh->dim != 1 && mesh->dim != 2) return DG_ERR_ARG;
    if (degree < 0 || degree > kMaxDeg) return DG_ERR_UNSUPPORTED;
    if (equation < 0 || equation > 2) return DG_ERR_ARG;
    if (opt->precision != DG_PREC_FP64 && opt->precision != DG_PREC_MIXED) return DG_ERR_ARG;
    if (opt->filter < 0 || opt->filter > 2) return DG_ERR_ARG;
    if (opt->quad_points != 0 && opt->quad_points != degree + 1) return DG_ERR_UNSUPPORTED;
    if (opt->positivity != 0 && opt->positivity != 1) return DG_ERR_ARG;
    if (opt->basis != 0 && opt->basis != 1) return DG_ERR_ARG;
    if (opt->cf_reading < 0 || opt->cf_reading > 2) return DG_ERR_ARG;
    if (opt->flux < DG_FLUX_LLF || opt->flux > DG_FLUX_HLLC) return DG_ERR_ARG;
    if (opt->flux != DG_FLUX_LLF && equation != DG_EQ_EULER) return DG_ERR_UNSUPPORTED;
    if (opt->positivity && equation != DG_EQ_EULER) return DG_ERR_UNSUPPORTED;
    if (!(opt->cfl > 0.0)) return DG_ERR_ARG;
    if (equation == DG_EQ_EULER && !(opt->gamma > 1.0)) return DG_ERR_ARG;
    for (int d = 0; d < mesh->dim; ++d) {
        if (mesh->n[d] < 1 || !(mesh->hi[d] > mesh->lo[d])) return DG_ERR_ARG;
        int b0 = mesh->bc[2 * d], b1 = mesh->bc[2 * d + 1];
        if (b0 < 0 || b0 > 5 || b1 < 0 || b1 > 5) return DG_ERR_ARG;
        if ((b0 == DG_BC_PERIODIC) != (b1 == DG_BC_PERIODIC)) return DG_ERR_ARG;
        if (mesh->dim == 1 && (b0 > 3 || b1 > 3)) return DG_ERR_ARG;
        if ((b0 == DG_BC_REFLECT || b1 == DG_BC_REFLECT) && equation != DG_EQ_EULER) return DG_ERR_ARG;
    }
    if (mesh->dim == 2) {
        if (equation == DG_EQ_BURGERS) return DG_ERR_UNSUPPORTED;
        for (int side = 0; side < 4; ++side) {
            const int b = mesh->bc[side];
            if ((b == DG_BC_DMR_WALL || b == DG_BC_DMR_TOP) && (side < 2 || equation != DG_EQ_EULER))
                return DG_ERR_ARG;
        }
    }
    dg_solver* s = new (std::nothrow) dg_solver;
    if (!s) return DG_ERR_ARG;
    memset(s, 0, sizeof *s);
    s->mesh = *mesh;
    s->opt = *opt;
    s->k = degree;
    s->eq = equation;
    s->dim = mesh->dim;
    s->nv = (equation == DG_EQ_EULER) ? (mesh->dim == 1 ? 3 : 4) : 1;
    // stored modes: P^k keeps the (k+1)(k+2)/2 modes p + q <= k (compact planes)
    s->pk = mesh->dim == 2 && opt->basis == 1 && degree > 0;
    s->nmodes = mesh->dim == 1 ? degree + 1
              : s->pk ? (degree + 1) * (degree + 2) / 2
                      : (degree + 1) * (degree + 1);
    s->lmax = mesh->dim == 1 ? degree : 2 * degree;
    s->ncell = mesh->dim == 1 ? mesh->n[0] : mesh->n[0] * mesh->n[1];
    s->n_pad = (s->ncell + 63) / 64 * 64;
    for (int d = 0; d < mesh->dim; ++d) {
        s->h[d] = (mesh->hi[d] - mesh->lo[d]) / (double)mesh->n[d];
        s->inv_h[d] = 1.0 / s->h[d];
    }
    if (opt->precision == DG_PREC_FP64)
        s->state_bytes = align256((size_t)s->nv * s->nmodes * s->ncell * sizeof(double));
    else
        s->state_bytes = align256((size_t)s->nv * s->n_pad * sizeof(double) +
                                  (size_t)s->nv * (s->nmodes - 1) * s->n_pad * sizeof(float));
    size_t off = kCtrlBytes;
    s->off_w = off;
    off += s->state_bytes;
    s->off_E = off;
    off += align256((size_t)s->ncell * (s->lmax + 1) * sizeof(double));
    s->off_eta = off;
    off += align256((size_t)s->ncell * sizeof(double));
    s->off_tcell = off;
    off += align256((size_t)s->ncell * sizeof(long long));
    s->off_tdata = off;
    off += align256((size_t)s->ncell * (s->lmax + 1) * sizeof(double));
    s->off_aux = off;
    off += kAuxBytes;
    // 2D positivity limiter: the cells a stage lists for it
    s->off_pcell = off;
    if (mesh->dim == 2 && opt->positivity) off += align256((size_t)s->ncell * sizeof(long long));
    // 2D hybrid runs: the stage output's corner values and the limiter
    // screen's verdicts, handed from the stage kernel to the indicator
    s->off_corner = s->off_ppfail = off;
    if (mesh->dim == 2 && opt->filter == DG_FILTER_HYBRID) {
        const size_t tb = opt->precision == DG_PREC_FP64 ? sizeof(double) : sizeof(float);
        off += align256((size_t)4 * s->nv * s->ncell * tb);
        s->off_ppfail = off;
        if (opt->positivity) off += align256((size_t)s->ncell);
    }
    s->off_dv = off;
    s->dv_slot = 0;
    if (mesh->dim == 1 && opt->filter == DG_FILTER_HYBRID && !opt->positivity) {
        const size_t tb = opt->precision == DG_PREC_FP64 ? sizeof(double) : sizeof(float);
        s->dv_slot = align256((size_t)s->ncell * (degree + 1) * tb);
        off += 4 * s->dv_slot;
    }
    s->ws_bytes = off;
    s->user_st = static_cast<hipStream_t>(opt->stream);
    if (hipStreamCreateWithFlags(&s->run_st, hipStreamNonBlocking) != hipSuccess) {
        delete s;
        return DG_ERR_DEVICE;
    }
    *out = s;
    return DG_OK;
}

int dg_destroy(dg_solver* s)
{
    if (!s) return DG_ERR_ARG;
    if (s->graph) (void)hipGraphExecDestroy(s->graph);
    if (s->run_st) (void)hipStreamDestroy(s->run_st);
    delete s;
    return DG_OK;
}

int dg_buffer_sizes(const dg_solver* s, size_t* state_bytes, size_t* workspace_bytes)
{
    if (!s) return DG_ERR_ARG;
    if (state_bytes) *state_bytes = s->state_bytes;
    if (workspace_bytes) *workspace_bytes = s->ws_bytes;
    return DG_OK;
}

int dg_bind(dg_solver* s, void* u_n, void* u_a, void* u_b, void* workspace)
{
    if (!s || !u_n || !u_a || !u_b || !workspace) return DG_ERR_ARG;
    void* ptrs[4] = {u_n, u_a, u_b, workspace};
    for (void* p : ptrs)
        if (((uintptr_t)p) & 255) return DG_ERR_ARG;
    if (u_n == u_a || u_n == u_b || u_a == u_b) return DG_ERR_ARG;
    s->u[0] = u_n;
    s->u[1] = u_a;
    s->u[2] = u_b;
    s->ws = static_cast<unsigned char*>(workspace);
    if (s->graph) {
        (void)hipGraphExecDestroy(s->graph);
        s->graph = nullptr;
    }
    Ctrl c;
    memset(&c, 0, sizeof c);
    c.dt_min = INFINITY;
    c.first_bad = -1;
    DG_HIP(hipStreamSynchronize(s->user_st));
    DG_HIP(hipMemcpy(workspace, &c, sizeof c, hipMemcpyHostToDevice));
    // deferred hybrid blend: no slot owes a blend until a stage writes it
    if (deferred_blend_on(s)) {
        const size_t tb = is_fp64(s) ? sizeof(double) : sizeof(float);
        for (int slot = 0; slot < 4; ++slot)
            DG_HIP(hipMemset(s->ws + s->off_dv + (size_t)slot * s->dv_slot, 0, s->ncell * tb));
    }
    s->bound = true;
    return DG_OK;
}

int dg_set_state(dg_solver* s, const double* modes_dev)
{
    if (!s || !modes_dev) return DG_ERR_ARG;
    if (!s->bound) return DG_ERR_STATE;
    if (s->pk) {
        if (is_fp64(s))
            DG_HIP(launch_convert_pk2d<double>(1, s->nv, s->k, s->ncell, modes_dev,
                                               view_of<double>(s, s->u[0]), s->user_st));
        else
            DG_HIP(launch_convert_pk2d<float>(1, s->nv, s->k, s->ncell, modes_dev,
                                              view_of<float>(s, s->u[0]), s->user_st));
    } else if (is_fp64(s)) {
        DG_HIP(hipMemcpyAsync(s->u[0], modes_dev, (size_t)s->nv * s->nmodes * s->ncell * sizeof(double),
                              hipMemcpyDeviceToDevice, s->user_st));
    } else {
        DG_HIP(launch_convert<float>(1, s->nv, s->nmodes, s->ncell, modes_dev,
                                     view_of<float>(s, s->u[0]), s->user_st));
    }
    return DG_OK;
}

int dg_get_state(dg_solver* s, double* modes_dev)
{
    if (!s || !modes_dev) return DG_ERR_ARG;
    if (!s->bound) return DG_ERR_STATE;
    if (s->pk) {
        if (is_fp64(s))
            DG_HIP(launch_convert_pk2d<double>(0, s->nv, s->k, s->ncell, modes_dev,
                                               view_of<double>(s, s->u[0]), s->user_st));
        else
            DG_HIP(launch_convert_pk2d<float>(0, s->nv, s->k, s->ncell, modes_dev,
                                              view_of<float>(s, s->u[0]), s->user_st));
    } else if (is_fp64(s)) {
        DG_HIP(hipMemcpyAsync(modes_dev, s->u[0], (size_t)s->nv * s->nmodes * s->ncell * sizeof(double),
                              hipMemcpyDeviceToDevice, s->user_st));
    } else {
        DG_HIP(launch_convert<float>(0, s->nv, s->nmodes, s->ncell, modes_dev,
                                     view_of<float>(s, s->u[0]), s->user_st));
    }
    return DG_OK;
}

int dg_max_wavespeed(dg_solver* s, double* alpha)
{
    if (!s || !alpha) return DG_ERR_ARG;
    if (!s->bound) return DG_ERR_STATE;
    double* aux = aux_of(s);
    unsigned long long* acc = reinterpret_cast<unsigned long long*>(aux + 10);
    DG_HIP(hipMemsetAsync(acc, 0, sizeof *acc, s->user_st));
    int rc = is_fp64(s) ? maxwave_impl<double>(s, acc, s->user_st) : maxwave_impl<float>(s, acc, s->user_st);
    if (rc) return rc;
    unsigned long long bits = 0;
    DG_HIP(hipMemcpyAsync(&bits, acc, sizeof bits, hipMemcpyDeviceToHost, s->user_st));
    DG_HIP(hipStreamSynchronize(s->user_st));
    memcpy(alpha, &bits, sizeof bits);
    return isfinite(*alpha) ? DG_OK : DG_ERR_NONFINITE;
}

int dg_stage(dg_solver* s, int stage, double dt)
{
    if (!s || stage < 0 || stage > 2 || !(dt >= 0.0)) return DG_ERR_ARG;
    if (!s->bound) return DG_ERR_STATE;
    return is_fp64(s) ? stage_impl<double>(s, stage, dt) : stage_impl<float>(s, stage, dt);
}

int dg_jump_filter(dg_solver* s, int stage, double dt)
{
    if (!s || stage < 0 || stage > 2 || !(dt >= 0.0)) return DG_ERR_ARG;
    if (!s->bound) return DG_ERR_STATE;
    return is_fp64(s) ? filter_impl<double>(s, stage, dt) : filter_impl<float>(s, stage, dt);
}

int dg_run(dg_solver* s, double t_end, int64_t max_steps, dg_report* rep)
{
    if (!s || max_steps < 0 || !(t_end == t_end)) return DG_ERR_ARG;
    if (!s->bound) return DG_ERR_STATE;
    return is_fp64(s) ? run_impl<double>(s, t_end, max_steps, rep)
                      : run_impl<float>(s, t_end, max_steps, rep);
}

int dg_report_read(dg_solver* s, dg_report* rep)
{
    if (!s) return DG_ERR_ARG;
    if (!s->bound) return DG_ERR_STATE;
    DG_HIP(hipStreamSynchronize(s->user_st));
    return is_fp64(s) ? report_impl<double>(s, rep) : report_impl<float>(s, rep);
}

int dg_time_kernel(dg_solver* s, int stage, double dt, int reps, double* avg_us)
{
    const int top = (s && s->dim == 2) ? 5 : 2;
    const bool step1d = s && s->dim == 1 && stage == 6;
    if (!s || stage < 0 || (stage > top && !step1d) || reps < 1 || !avg_us || !(dt >= 0.0))
        return DG_ERR_ARG;
    if (!s->bound) return DG_ERR_STATE;
    DG_HIP(hipStreamSynchronize(s->user_st));
    return is_fp64(s) ? time_impl<double>(s, stage, dt, reps, avg_us)
                      : time_impl<float>(s, stage, dt, reps, avg_us);
}

int dg_max_wavespeed_noalloc(const dg_solver* s, const void* u_dev, double* alpha, int64_t* first_bad)
{
    if (!s || !u_dev || !alpha) return DG_ERR_ARG;
    if (s->ncell > (int64_t)kNoallocBlocks * 256) return DG_ERR_ARG;
    NoallocScratch* sc = noalloc_scratch();
    if (!sc) return DG_ERR_DEVICE;
    // mode 0 of variable v of the state buffer: FP64 layout v * nmodes * ncell;
    // mixed layout v * n_pad (the planes of mode 0 come first)
    const double* m0 = static_cast<const double*>(u_dev);
    const int64_t s0 = s->opt.precision == DG_PREC_FP64 ? (int64_t)s->nmodes * s->ncell : s->n_pad;
    PhysParams ph;
    memset(&ph, 0, sizeof ph);
    ph.gamma = s->opt.gamma;
    ph.flux = s->opt.flux;
    ph.a[0] = s->opt.adv_speed[0];
    ph.a[1] = s->opt.adv_speed[1];
    const double ihx = s->inv_h[0], ihy = s->dim == 2 ? s->inv_h[1] : 0.0;
    hipStream_t st = s->user_st;
    hipError_t e = hipErrorInvalidValue;
    if (s->dim == 1)
        e = s->eq == DG_EQ_EULER    ? launch_noalloc<EULER, 1>(m0, s0, s->ncell, ph, ihx, ihy, sc, st)
          : s->eq == DG_EQ_BURGERS ? launch_noalloc<BURGERS, 1>(m0, s0, s->ncell, ph, ihx, ihy, sc, st)
                                   : launch_noalloc<ADV, 1>(m0, s0, s->ncell, ph, ihx, ihy, sc, st);
    else
        e = s->eq == DG_EQ_EULER ? launch_noalloc<EULER, 2>(m0, s0, s->ncell, ph, ihx, ihy, sc, st)
                                 : launch_noalloc<ADV, 2>(m0, s0, s->ncell, ph, ihx, ihy, sc, st);
    if (e != hipSuccess) return DG_ERR_DEVICE;
    struct {
        double alpha;
        long long first_bad;
        int status;
    } r;
    DG_HIP(hipMemcpyAsync(&r.alpha, &sc->alpha, sizeof(double), hipMemcpyDeviceToHost, st));
    DG_HIP(hipMemcpyAsync(&r.first_bad, &sc->first_bad, sizeof(long long), hipMemcpyDeviceToHost, st));
    DG_HIP(hipMemcpyAsync(&r.status, &sc->status, sizeof(int), hipMemcpyDeviceToHost, st));
    DG_HIP(hipStreamSynchronize(st));
    *alpha = r.alpha;
    if (first_bad) *first_bad = r.status ? r.first_bad : -1;
    return isfinite(*alpha) ? DG_OK : DG_ERR_NONFINITE;
}

int dg_last_exponents(dg_solver* s, double* E_dev)
{
    if (!s || !E_dev) return DG_ERR_ARG;
    if (!s->bound) return DG_ERR_STATE;
    DG_HIP(hipMemcpyAsync(E_dev, s->ws + s->off_E, (size_t)s->ncell * (s->lmax + 1) * sizeof(double),
                          hipMemcpyDeviceToDevice, s->user_st));
    return DG_OK;
}

}  // extern "C"
