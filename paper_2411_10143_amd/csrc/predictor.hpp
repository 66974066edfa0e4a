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

struct Cascade {
    Tree tree[3];   // format, algorithm, lanes
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

}  // namespace ck
