// dg_batch.h — argument and report blocks of the batched 1D launch.
#pragma once

#include "dg_kernels.h"

namespace dg {

struct BatchProb {
    long long n, n_pad;     // cells, padded plane length
    long long off_ext;      // element offset of the FP64 exchange-layout state
    long long off_int;      // byte offset of the problem's block in each state buffer
    double lo, h, inv_h;
    double t_end;
    int k, bc_lo, bc_hi, pad;
};

struct BatchReport {
    long long steps;
    double t, dt_min, dt_max;
    double ledger[3], bflux[3];
    int status, pad;
    long long first_bad;
    long long restarts;     // steps retried with half dt (positivity limiter)
};

struct BatchArgs {
    void* u[3];             // three state buffers (internal layout)
    const BatchProb* probs;
    const unsigned int* order;  // queue order (longest first)
    unsigned int* queue;        // next queue position
    Ctrl* ctrl;                 // per-problem error latch
    BatchReport* report;
    int nprob;
    long long steps;
    double cfl;
    PhysParams phys;
    int pp;                 // positivity-preserving limiter after the filter
};

// bs: threads per workgroup, 128 or 256 (tiles of bs - 12 cells)
hipError_t launch_batch1d(int mixed, int mode, const BatchArgs& b, int grid, int bs, hipStream_t st);
hipError_t launch_batch_reset(const BatchArgs& b, hipStream_t st);
template <typename TB>
hipError_t launch_batch_convert(int to_internal, const BatchArgs& b, const double* ext, int nprob,
                                hipStream_t st);

}  // namespace dg
