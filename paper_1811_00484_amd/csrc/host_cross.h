// Tucker cross approximation of one defining tensor from an entry callback
// (host, FP64); see host_cross.cpp for the scheme.
#pragma once
#include <string>

#include "host_compress.h"
#include "vie.h"

namespace vie {

struct CrossParams {
    double tol = 1e-6;
    int rule = 0;
    int max_rank = 0;
    int oversample = 8;
    int start = 2;
    int max_sweeps = 8;
    int n_sample = 0;
    unsigned long long seed = 0;
};

struct CrossStats {
    long evals = 0;          // entries requested to build the form
    long evals_sample = 0;   // entries requested for the error estimate
    int sweeps = 0;
    int cross_ranks[3] = {0, 0, 0};
    double sample_rel_err = 0;
};

// 0 on success; -1 callback error, -4 non-finite entry, -5 numerical failure
// or max_rank too small (message in err).  odd[a]: the component vanishes at
// offset 0 along axis a (those entries are taken as exact zeros).
int tucker_cross(vie_entry_fn fn, void* ctx, int comp, const int odd[3], const int n[3], const CrossParams& p,
                 TuckerComponent& out, CrossStats& st, std::string& err);

}  // namespace vie
