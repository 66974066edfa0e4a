// Cascaded SpMV-configuration predictor (Section III-C-1, cascaded-prediction
// figure): three decision trees evaluated in sequence.
//   stage 1 "format"    : CSR / ELL / COO / DIA / HYB
//   stage 2 "algorithm" : (CSR only) scalar / vector / merge-path / panel
//   stage 3 "lanes"     : (CSR-vector only) log2 of lanes per row, 0..6
// and optionally a "start" tree over the inputs known before any pass over
// the entries (dimensions, nnz, density, mean row length), which picks the
// configuration a solve starts from among those that need no copy of the
// matrix (a known-features-only first stage, from the related work the
// paper discusses, Sections II-B and V).
// The paper compiles its trained models to C with m2cgen so inference costs
// microseconds instead of milliseconds (inference-time table); here each tree
// is a flat node table walked by a few lines of C++.
//
// Model file (text): comment lines start with '#'; each tree is
//   tree <name> <node count>
// followed by one line per node:
//   <feature index or -1 for a leaf> <threshold, C99 hex float> <left> <right> <class>
// An internal node sends a feature vector left iff (double)(float)f[feature]
// <= threshold (the tree was fitted on single-precision inputs).
#include <dlfcn.h>

#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "derive.hpp"
#include "predictor.hpp"

namespace ck {

namespace {

std::mutex g_models_mu;
std::map<std::string, Cascade> g_models;

bool parse_model(const std::string &path, Cascade &out, std::string &err) {
    FILE *f = fopen(path.c_str(), "r");
    if (!f) {
        err = "cannot open cascade model '" + path + "'";
        return false;
    }
    char line[512];
    Tree *cur = nullptr;
    int expect = 0;
    bool ok = true;
    while (ok && fgets(line, sizeof line, f)) {
        if (line[0] == '#' || line[0] == '\n')
            continue;
        if (strncmp(line, "tree ", 5) == 0) {
            char name[64];
            int count = 0;
            if (sscanf(line + 5, "%63s %d", name, &count) != 2 || count <= 0) {
                ok = false;
                break;
            }
            if (!strcmp(name, "format"))
                cur = &out.tree[0];
            else if (!strcmp(name, "algorithm"))
                cur = &out.tree[1];
            else if (!strcmp(name, "lanes"))
                cur = &out.tree[2];
            else if (!strcmp(name, "start")) {
                cur = &out.start;
                out.has_start = true;
            } else {
                ok = false;
                break;
            }
            cur->feature.clear();
            cur->threshold.clear();
            cur->left.clear();
            cur->right.clear();
            cur->cls.clear();
            expect = count;
            continue;
        }
        if (!cur || expect <= 0) {
            ok = false;
            break;
        }
        int fe, le, ri, cl;
        char thr[128];
        if (sscanf(line, "%d %127s %d %d %d", &fe, thr, &le, &ri, &cl) != 5) {
            ok = false;
            break;
        }
        cur->feature.push_back(fe);
        cur->threshold.push_back(strtod(thr, nullptr));
        cur->left.push_back(le);
        cur->right.push_back(ri);
        cur->cls.push_back(cl);
        --expect;
    }
    fclose(f);
    if (ok) {
        // classes per stage: format 0..4, CSR algorithm 0..3, log2(lanes)
        // 0..6; the start tree: configuration ids 0..8 on the known inputs
        static const int kClasses[4] = {5, 4, 7, 9};
        static const int kInputs[4] = {kNumModelFeatures, kNumModelFeatures,
                                       kNumModelFeatures, kNumKnownFeatures};
        for (int t = 0; t < 4 && ok; ++t) {
            if (t == 3 && !out.has_start)
                break;
            const Tree &T = t < 3 ? out.tree[t] : out.start;
            const int nn = (int)T.feature.size();
            if (nn == 0)
                ok = false;
            for (int i = 0; i < nn && ok; ++i) {
                if (T.feature[i] >= 0 &&
                    (T.feature[i] >= kInputs[t] || T.left[i] <= i || T.right[i] <= i ||
                     T.left[i] >= nn || T.right[i] >= nn))
                    ok = false;   // children come after parents: the walk ends
                if (T.feature[i] < 0 && (T.cls[i] < 0 || T.cls[i] >= kClasses[t]))
                    ok = false;   // a leaf names a class the stage does not have
            }
        }
    }
    if (!ok)
        err = "malformed cascade model '" + path + "'";
    return ok;
}

std::string default_model_path() {
    const char *env = std::getenv("CK_CASCADE_MODEL");
    if (env && *env)
        return std::string(env);
    Dl_info info;
    if (dladdr((void *)&default_model_path, &info) && info.dli_fname) {
        std::string p(info.dli_fname);
        const size_t slash = p.rfind('/');
        return (slash == std::string::npos ? std::string(".") : p.substr(0, slash)) +
               "/cascade_model.txt";
    }
    return "cascade_model.txt";
}

}  // namespace

const Cascade *load_cascade(const char *path, std::string &err) {
    const std::string key = path ? std::string(path) : default_model_path();
    std::lock_guard<std::mutex> lk(g_models_mu);
    auto it = g_models.find(key);
    if (it != g_models.end())
        return &it->second;
    Cascade c;
    if (!parse_model(key, c, err))
        return nullptr;
    return &g_models.emplace(key, std::move(c)).first->second;
}

int Tree::eval(const double *f) const {
    int t = 0;
    while (feature[t] >= 0) {
        const double v = (double)(float)f[feature[t]];
        t = v <= threshold[t] ? left[t] : right[t];
    }
    return cls[t];
}

static_assert(offsetof(ck_features, density) == 28 * sizeof(int64_t),
              "the 28 integer fields of ck_features come first, in order");

// The floating-point features from the integer ones (derive.hpp: the same
// derivation as the device-resident cascade's).
void derive_features(ck_features &F) {
    int64_t I[28];
    std::memcpy(I, &F, sizeof I);
    double d[9];
    derive_inputs(I, d);
    F.density = d[0];
    F.mean = d[1];
    F.sd = d[2];
    F.cov = d[3];
    F.maxavg = d[4];
    F.distavg = d[5];
    F.clusteravg = d[6];
    F.fill = d[7];
    F.diagfill = d[8];
}

// The 15 model inputs in feature-table order.
void model_inputs(const ck_features &F, double *f) {
    int64_t I[28];
    std::memcpy(I, &F, sizeof I);
    const double d[9] = {F.density, F.mean, F.sd, F.cov, F.maxavg, F.distavg, F.clusteravg,
                         F.fill, F.diagfill};
    model_inputs_from(I, d, f);
}

int start_config_id(const Cascade &C, int64_t nrows, int64_t ncols, int64_t nnz) {
    if (!C.has_start)
        return -1;
    // the same derivation as for the full feature set, from dimensions only
    ck_features F{};
    F.nrows = nrows;
    F.ncols = ncols;
    F.nnz = nnz;
    derive_features(F);
    double in[kNumModelFeatures];
    model_inputs(F, in);
    return C.start.eval(in);
}

ck_config stage_config(int stage, int cls, const ck_config &prev) {
    ck_config c = prev;
    if (stage == 0) {
        c.format = cls;
        if (cls != CK_FMT_CSR) {
            c.algorithm = 0;
            c.lanes = 0;
        }
    } else if (stage == 1) {
        c.algorithm = cls;
        if (cls != CK_ALG_VECTOR)
            c.lanes = 0;
    } else {
        c.lanes = 1 << cls;
    }
    c.stages_done = stage + 1;
    return c;
}

}  // namespace ck
