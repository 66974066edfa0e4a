// Cascaded decision-tree predictor (host side).
#pragma once

#include <string>
#include <vector>

#include "../../include/caskrylov.h"

namespace ck {

constexpr int kNumModelFeatures = 15;

struct Tree {
    std::vector<int> feature, left, right, cls;
    std::vector<double> threshold;
    int eval(const double *f) const;
};

// Inputs 0..4 of the feature table (nrows, ncols, nnz, density, mean) follow
// from the matrix's dimensions alone, without a pass over its entries.
constexpr int kNumKnownFeatures = 5;

struct Cascade {
    Tree tree[3];   // format, algorithm, lanes
    // optional starting configuration from the known inputs alone: a
    // configuration id 0..8 (the CSR configurations that need no copy)
    Tree start;
    bool has_start = false;
};

// Loads (once, then cached) a model file; NULL path = the model shipped next
// to the library.  Returns nullptr and sets err on failure.
const Cascade *load_cascade(const char *path, std::string &err);

// Fills the floating-point fields of F from its integer accumulators.
void derive_features(ck_features &F);
// The 15 model inputs in feature-table order.
void model_inputs(const ck_features &F, double *f);
// The configuration after a stage decision `cls` applied to `prev`.
ck_config stage_config(int stage, int cls, const ck_config &prev);
// The starting configuration id the cascade's start tree gives for a matrix
// of these dimensions, or -1 if the model has none.
int start_config_id(const Cascade &C, int64_t nrows, int64_t ncols, int64_t nnz);

}  // namespace ck
