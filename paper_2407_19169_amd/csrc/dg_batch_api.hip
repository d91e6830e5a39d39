// dg_batch_api.hip — host side of the batched 1D ABI (include/dg.h) and
// its autotuner.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <numeric>
#include <vector>

#include "../../include/dg.h"
#include "dg_batch.h"

using namespace dg;

struct dg_batch {
    int nprob, eq;
    dg_options opt;
    std::vector<BatchProb> probs;
    std::vector<unsigned int> order_lpt, order_natural;
    size_t state_bytes, ws_bytes;
    size_t off_probs, off_order, off_queue, off_ctrl, off_report, off_backup;
    void* u[3];
    unsigned char* ws;
    bool bound;
    hipStream_t st;      // the caller's stream
    hipStream_t run_st;  // private stream the run's graph is captured on and replayed
    hipGraphExec_t graph;
    long long graph_steps;
    int graph_grid, graph_bs;
    BatchReport* host_rep;  // pinned host copy of the per-problem reports
    int grid;          // persistent workgroups
    int bs;            // threads per workgroup (128 or 256)
    int use_lpt;       // queue order
    int cus;           // compute units of the device
};

namespace {

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

#define DG_HIP(call)                                \
    do {                                            \
        hipError_t e_ = (call);                     \
        if (e_ != hipSuccess) return DG_ERR_DEVICE; \
    } while (0)

BatchArgs batch_args(const dg_batch* b, long long steps)
{
    BatchArgs a;
    memset(&a, 0, sizeof a);
    for (int i = 0; i < 3; ++i) a.u[i] = b->u[i];
    a.probs = reinterpret_cast<const BatchProb*>(b->ws + b->off_probs);
    a.order = reinterpret_cast<const unsigned int*>(b->ws + b->off_order);
    a.queue = reinterpret_cast<unsigned int*>(b->ws + b->off_queue);
    a.ctrl = reinterpret_cast<Ctrl*>(b->ws + b->off_ctrl);
    a.report = reinterpret_cast<BatchReport*>(b->ws + b->off_report);
    a.nprob = b->nprob;
    a.steps = steps;
    a.cfl = b->opt.cfl;
    a.pp = b->opt.positivity;
    a.phys.gamma = b->opt.gamma;
    return a;
}

int upload_order(dg_batch* b, int lpt)
{
    const std::vector<unsigned int>& o = lpt ? b->order_lpt : b->order_natural;
    DG_HIP(hipMemcpy(b->ws + b->off_order, o.data(), o.size() * sizeof(unsigned int),
                     hipMemcpyHostToDevice));
    b->use_lpt = lpt;
    return DG_OK;
}

// Clear the queue head and the per-problem error latches (a kernel, so the
// run can be captured in a graph).
int reset_run(dg_batch* b, hipStream_t st)
{
    DG_HIP(launch_batch_reset(batch_args(b, 0), st));
    return DG_OK;
}

int launch(dg_batch* b, long long steps, hipStream_t st)
{
    const int mode = b->opt.filter == DG_FILTER_NONE ? 0 : 1;
    DG_HIP(launch_batch1d(b->opt.precision == DG_PREC_MIXED, mode, batch_args(b, steps), b->grid, b->bs, st));
    return DG_OK;
}

void drop_graph(dg_batch* b)
{
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
}

// The run as one graph on the private stream: reset, the persistent launch,
// and the copy of the reports into pinned host memory.  Kept while the step
// count and the schedule stay the same.
int run_graph(dg_batch* b, long long steps)
{
    if (b->graph && (b->graph_steps != steps || b->graph_grid != b->grid || b->graph_bs != b->bs))
        drop_graph(b);
    if (!b->graph) {
        hipGraph_t g = nullptr;
        DG_HIP(hipStreamBeginCapture(b->run_st, hipStreamCaptureModeThreadLocal));
        int rc = reset_run(b, b->run_st);
        if (!rc) rc = launch(b, steps, b->run_st);
        if (!rc && hipMemcpyAsync(b->host_rep, b->ws + b->off_report, sizeof(BatchReport) * b->nprob,
                                  hipMemcpyDeviceToHost, b->run_st) != hipSuccess)
            rc = DG_ERR_DEVICE;
        const hipError_t e = hipStreamEndCapture(b->run_st, &g);
        if (rc || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return rc ? rc : DG_ERR_DEVICE;
        }
        const hipError_t ei = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) {
            b->graph = nullptr;
            return DG_ERR_DEVICE;
        }
        b->graph_steps = steps;
        b->graph_grid = b->grid;
        b->graph_bs = b->bs;
    }
    DG_HIP(hipGraphLaunch(b->graph, b->run_st));
    DG_HIP(hipStreamSynchronize(b->run_st));
    return DG_OK;
}

}  // namespace

extern "C" {

int dg_batch_create(int nprob, dg_problem1d* probs, int equation, const dg_options* opt,
                    int64_t* total_elems, dg_batch** out)
{
    if (!out) return DG_ERR_ARG;
    *out = nullptr;
    if (nprob < 1 || !probs || !opt || !total_elems) return DG_ERR_ARG;
    if (equation != DG_EQ_EULER) return DG_ERR_UNSUPPORTED;
    if (opt->filter == DG_FILTER_HYBRID) return DG_ERR_UNSUPPORTED;
    if (opt->positivity != 0 && opt->positivity != 1) return DG_ERR_ARG;
    if (opt->basis != 0 && opt->basis != 1) return DG_ERR_ARG;  // 1D: the same space
    if (opt->flux < DG_FLUX_LLF || opt->flux > DG_FLUX_HLLC) return DG_ERR_ARG;
    if (opt->flux != DG_FLUX_LLF) return DG_ERR_UNSUPPORTED;
    if (opt->precision != DG_PREC_FP64 && opt->precision != DG_PREC_MIXED) return DG_ERR_ARG;
    if (!(opt->cfl > 0.0) || !(opt->gamma > 1.0)) return DG_ERR_ARG;
    dg_batch* b = new (std::nothrow) dg_batch();
    if (!b) return DG_ERR_ARG;
    b->nprob = nprob;
    b->eq = equation;
    b->opt = *opt;
    b->probs.resize(nprob);
    long long ext = 0;
    size_t off = 0;
    for (int i = 0; i < nprob; ++i) {
        const dg_problem1d& p = probs[i];
        const bool per = p.bc[0] == DG_BC_PERIODIC, per1 = p.bc[1] == DG_BC_PERIODIC;
        if (p.n < 1 || p.degree < 0 || p.degree > 3 || !(p.hi > p.lo) || per != per1 || p.bc[0] < 0 ||
            p.bc[0] > 2 || p.bc[1] < 0 || p.bc[1] > 2) {
            delete b;
            return p.degree > 3 ? DG_ERR_UNSUPPORTED : DG_ERR_ARG;
        }
        BatchProb& q = b->probs[i];
        memset(&q, 0, sizeof q);
        q.n = p.n;
        q.n_pad = (p.n + 63) / 64 * 64;
        q.k = p.degree;
        q.bc_lo = p.bc[0];
        q.bc_hi = p.bc[1];
        q.lo = p.lo;
        q.h = (p.hi - p.lo) / (double)p.n;
        q.inv_h = 1.0 / q.h;
        q.t_end = INFINITY;
        q.off_ext = ext;
        probs[i].offset = ext;
        ext += 3LL * (p.degree + 1) * p.n;
        q.off_int = (long long)off;
        const size_t bytes = opt->precision == DG_PREC_FP64
                                 ? 3 * (size_t)(p.degree + 1) * q.n_pad * 8
                                 : 3 * (size_t)q.n_pad * 8 + 3 * (size_t)p.degree * q.n_pad * 4;
        off += a256(bytes);
    }
    *total_elems = ext;
    b->state_bytes = a256(off);
    size_t w = 0;
    b->off_probs = w;
    w += a256(sizeof(BatchProb) * nprob);
    b->off_order = w;
    w += a256(sizeof(unsigned int) * nprob);
    b->off_queue = w;
    w += 256;
    b->off_ctrl = w;
    w += a256(sizeof(Ctrl) * nprob);
    b->off_report = w;
    w += a256(sizeof(BatchReport) * nprob);
    b->off_backup = w;
    w += b->state_bytes;
    b->ws_bytes = w;
    // longest-processing-time-first queue: cost ~ n (k+1)^2
    b->order_natural.resize(nprob);
    std::iota(b->order_natural.begin(), b->order_natural.end(), 0u);
    b->order_lpt = b->order_natural;
    std::stable_sort(b->order_lpt.begin(), b->order_lpt.end(), [&](unsigned x, unsigned y) {
        const double cx = (double)b->probs[x].n * (b->probs[x].k + 1) * (b->probs[x].k + 1);
        const double cy = (double)b->probs[y].n * (b->probs[y].k + 1) * (b->probs[y].k + 1);
        return cx > cy;
    });
    int dev = 0;
    hipDeviceProp_t prop;
    b->cus = 256;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        b->cus = prop.multiProcessorCount;
    b->grid = 2 * b->cus;
    b->bs = 256;
    b->use_lpt = 1;
    b->st = static_cast<hipStream_t>(opt->stream);
    if (hipStreamCreateWithFlags(&b->run_st, hipStreamNonBlocking) != hipSuccess) {
        delete b;
        return DG_ERR_DEVICE;
    }
    if (hipHostMalloc(reinterpret_cast<void**>(&b->host_rep), sizeof(BatchReport) * nprob,
                      hipHostMallocDefault) != hipSuccess) {
        (void)hipStreamDestroy(b->run_st);
        delete b;
        return DG_ERR_DEVICE;
    }
    *out = b;
    return DG_OK;
}

int dg_batch_destroy(dg_batch* b)
{
    if (!b) return DG_ERR_ARG;
    drop_graph(b);
    if (b->run_st) (void)hipStreamDestroy(b->run_st);
    if (b->host_rep) (void)hipHostFree(b->host_rep);
    delete b;
    return DG_OK;
}

int dg_batch_buffer_sizes(const dg_batch* b, size_t* state_bytes, size_t* workspace_bytes)
{
    if (!b) return DG_ERR_ARG;
    if (state_bytes) *state_bytes = b->state_bytes;
    if (workspace_bytes) *workspace_bytes = b->ws_bytes;
    return DG_OK;
}

int dg_batch_bind(dg_batch* b, void* u_n, void* u_a, void* u_b, void* workspace)
{
    if (!b || !u_n || !u_a || !u_b || !workspace) return DG_ERR_ARG;
    void* ptrs[4] = {u_n, u_a, u_b, workspace};
    for (void* p : ptrs)
        if (((uintptr_t)p) & 255) return DG_ERR_ARG;
    b->u[0] = u_n;
    b->u[1] = u_a;
    b->u[2] = u_b;
    b->ws = static_cast<unsigned char*>(workspace);
    drop_graph(b);
    DG_HIP(hipStreamSynchronize(b->st));
    DG_HIP(hipMemcpy(b->ws + b->off_probs, b->probs.data(), sizeof(BatchProb) * b->nprob,
                     hipMemcpyHostToDevice));
    int rc = upload_order(b, b->use_lpt);
    if (rc) return rc;
    DG_HIP(hipMemset(b->ws + b->off_report, 0, sizeof(BatchReport) * b->nprob));
    b->bound = true;
    return DG_OK;
}

int dg_batch_set_state(dg_batch* b, const double* packed_dev)
{
    if (!b || !packed_dev) return DG_ERR_ARG;
    if (!b->bound) return DG_ERR_STATE;
    const BatchArgs a = batch_args(b, 0);
    if (b->opt.precision == DG_PREC_MIXED)
        DG_HIP(launch_batch_convert<float>(1, a, packed_dev, b->nprob, b->st));
    else
        DG_HIP(launch_batch_convert<double>(1, a, packed_dev, b->nprob, b->st));
    return DG_OK;
}

int dg_batch_get_state(dg_batch* b, double* packed_dev)
{
    if (!b || !packed_dev) return DG_ERR_ARG;
    if (!b->bound) return DG_ERR_STATE;
    const BatchArgs a = batch_args(b, 0);
    if (b->opt.precision == DG_PREC_MIXED)
        DG_HIP(launch_batch_convert<float>(0, a, packed_dev, b->nprob, b->st));
    else
        DG_HIP(launch_batch_convert<double>(0, a, packed_dev, b->nprob, b->st));
    return DG_OK;
}

int dg_batch_run(dg_batch* b, const double* t_end, int64_t steps, dg_report* per_problem)
{
    if (!b || steps < 0) return DG_ERR_ARG;
    if (!b->bound) return DG_ERR_STATE;
    DG_HIP(hipStreamSynchronize(b->st));
    if (t_end) {
        for (int i = 0; i < b->nprob; ++i) b->probs[i].t_end = t_end[i];
        DG_HIP(hipMemcpy(b->ws + b->off_probs, b->probs.data(), sizeof(BatchProb) * b->nprob,
                         hipMemcpyHostToDevice));
    }
    const int rc = run_graph(b, steps);
    if (rc) return rc;
    const BatchReport* rep = b->host_rep;
    int status = DG_OK;
    for (int i = 0; i < b->nprob; ++i) {
        if (rep[i].status && status == DG_OK) status = rep[i].status;
        if (!per_problem) continue;
        dg_report& r = per_problem[i];
        memset(&r, 0, sizeof r);
        r.steps = rep[i].steps;
        r.t = rep[i].t;
        r.dt_min = rep[i].dt_min;
        r.dt_max = rep[i].dt_max;
        for (int v = 0; v < 3; ++v) {
            r.ledger[v] = rep[i].ledger[v];
            r.boundary_flux[v] = rep[i].bflux[v];
        }
        r.min_rho = r.min_p = r.max_exponent = NAN;
        r.status = rep[i].status;
        r.first_bad_cell = rep[i].status ? rep[i].first_bad : -1;
        r.restarts = rep[i].restarts;
    }
    return status;
}

// Autotuner: times `trial_steps` steps of the whole batch for every
// candidate schedule (threads per workgroup 256 or 128, i.e. tiles of 244 or
// 116 cells; persistent workgroups per compute unit; queue order), each from
// the same saved state, keeps the fastest, restores the state and writes a
// JSON summary to json (nullable, capacity cap) with the key of the batch's
// shape: the fractions of P0..P3 problems and the size bucket
// round(log2(mean cells)).
int dg_batch_tune(dg_batch* b, int64_t trial_steps, char* json, size_t cap)
{
    if (!b || trial_steps < 1) return DG_ERR_ARG;
    if (!b->bound) return DG_ERR_STATE;
    DG_HIP(hipStreamSynchronize(b->st));
    DG_HIP(hipMemcpy(b->ws + b->off_backup, b->u[0], b->state_bytes, hipMemcpyDeviceToDevice));
    const int factors[4] = {1, 2, 4, 8};
    const int sizes[2] = {256, 128};
    struct Cand {
        int bs, factor, lpt;
        float ms;
    };
    std::vector<Cand> cands;
    hipEvent_t e0, e1;
    DG_HIP(hipEventCreate(&e0));
    DG_HIP(hipEventCreate(&e1));
    int rc = DG_OK;
    for (int lpt = 1; lpt >= 0 && rc == DG_OK; --lpt) {
        rc = upload_order(b, lpt);
        for (int sz = 0; sz < 2 && rc == DG_OK; ++sz)
            for (int f = 0; f < 4 && rc == DG_OK; ++f) {
                b->bs = sizes[sz];
                // a 128-thread workgroup is half a 256-thread one: twice as
                // many fill the same compute unit
                const int per_cu = factors[f] * (256 / b->bs);
                b->grid = per_cu * b->cus;
                if (hipMemcpyAsync(b->u[0], b->ws + b->off_backup, b->state_bytes,
                                   hipMemcpyDeviceToDevice, b->st) != hipSuccess)
                    rc = DG_ERR_DEVICE;
                if (!rc) rc = reset_run(b, b->st);
                if (!rc && hipEventRecord(e0, b->st) != hipSuccess) rc = DG_ERR_DEVICE;
                if (!rc) rc = launch(b, trial_steps, b->st);
                if (!rc && hipEventRecord(e1, b->st) != hipSuccess) rc = DG_ERR_DEVICE;
                if (!rc && hipEventSynchronize(e1) != hipSuccess) rc = DG_ERR_DEVICE;
                float ms = 0.f;
                if (!rc && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = DG_ERR_DEVICE;
                cands.push_back({sizes[sz], per_cu, lpt, ms});
            }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (hipMemcpy(b->u[0], b->ws + b->off_backup, b->state_bytes, hipMemcpyDeviceToDevice) != hipSuccess)
        rc = DG_ERR_DEVICE;
    if (rc) return rc;
    const Cand* best = &cands[0];
    for (const Cand& c : cands)
        if (c.ms < best->ms) best = &c;
    b->bs = best->bs;
    b->grid = best->factor * b->cus;
    rc = upload_order(b, best->lpt);
    if (json && cap) {
        double kf[4] = {0, 0, 0, 0}, mean_n = 0.0;
        for (const BatchProb& q : b->probs) {
            kf[q.k] += 1.0 / b->nprob;
            mean_n += (double)q.n / b->nprob;
        }
        size_t used = 0;
        auto put = [&](const char* fmt, auto... args) {
            if (used < cap) {
                int w = snprintf(json + used, cap - used, fmt, args...);
                if (w > 0) used += (size_t)w;
            }
        };
        put("{\"key\": {\"k_mix\": [%.2f, %.2f, %.2f, %.2f], \"n_bucket\": %d}, \"trial_steps\": %lld, "
            "\"candidates\": [",
            kf[0], kf[1], kf[2], kf[3], (int)lround(log2(mean_n > 1.0 ? mean_n : 1.0)),
            (long long)trial_steps);
        for (size_t i = 0; i < cands.size(); ++i)
            put("%s{\"block_size\": %d, \"wg_per_cu\": %d, \"order\": \"%s\", \"ms\": %.4f}", i ? ", " : "",
                cands[i].bs, cands[i].factor, cands[i].lpt ? "lpt" : "natural", cands[i].ms);
        put("], \"best\": {\"block_size\": %d, \"wg_per_cu\": %d, \"order\": \"%s\", \"ms\": %.4f}}",
            best->bs, best->factor, best->lpt ? "lpt" : "natural", best->ms);
    }
    return rc;
}

int dg_batch_set_schedule(dg_batch* b, int block_size, int wg_per_cu, int lpt)
{
    if (!b || (block_size != 128 && block_size != 256) || wg_per_cu < 1 || wg_per_cu > 16 ||
        (lpt != 0 && lpt != 1))
        return DG_ERR_ARG;
    if (!b->bound) return DG_ERR_STATE;
    DG_HIP(hipStreamSynchronize(b->st));
    b->bs = block_size;
    b->grid = wg_per_cu * b->cus;
    return upload_order(b, lpt);
}

}  // extern "C"
