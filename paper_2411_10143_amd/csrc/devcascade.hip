// Device-resident cascade: the three-stage prediction of Section III-C-1
// (cascaded-prediction figure) evaluated on the GPU, after the feature pass,
// with no host round trip in between.  The paper evaluates its trees on the
// host (compiled to C so that inference costs microseconds, inference-time
// table of Section III-C-2); here the feature accumulators never leave the
// device: one thread derives the 15 model inputs (derive.hpp, the same
// derivation the host cascade uses) and walks the format, algorithm and
// lanes trees, stream-ordered behind the feature kernels.
#include <map>
#include <mutex>

#include "derive.hpp"
#include "matrix.hpp"
#include "predictor.hpp"

namespace ck {

int64_t features_scratch_bytes(int64_t n, int64_t ncols, int64_t nnz);
ck_status launch_features(const ck_matrix &M, void *scratch, bool symmetry, hipStream_t s);
ck_status launch_feature_ints(const ck_matrix &M, const void *scratch, bool symmetry,
                              int64_t *out28, hipStream_t s);

namespace {

// One tree's node table in device memory.
struct DevTree {
    const int *feature, *left, *right, *cls;
    const double *thr;
};
struct DevModel {
    DevTree t[3];   // format, algorithm, lanes
};

__device__ int walk(const DevTree &T, const double *f) {
    int k = 0;
    while (T.feature[k] >= 0) {
        const double v = (double)(float)f[T.feature[k]];
        k = v <= T.thr[k] ? T.left[k] : T.right[k];
    }
    return T.cls[k];
}

// ck_config_id of a cascade outcome (format, algorithm, log2 lanes)
__device__ int config_id_of(int fmt, int alg, int lanes) {
    if (fmt == CK_FMT_ELL)
        return 9;
    if (fmt == CK_FMT_COO)
        return 10;
    if (fmt == CK_FMT_DIA)
        return 12;
    if (fmt == CK_FMT_HYB)
        return 13;
    if (alg == CK_ALG_SCALAR)
        return 7;
    if (alg == CK_ALG_MERGE)
        return 8;
    if (alg == CK_ALG_PANEL)
        return 11;
    int idx = 0;
    while ((1 << idx) < lanes)
        ++idx;
    return idx;
}

// The cascade for one matrix: stage 1 the format; stage 2 the CSR
// algorithm, only for CSR; stage 3 the lanes, only for CSR-vector.  A stage
// that does not run keeps the default configuration's field (CSR-vector
// with clamp(2^floor(log2(max(1, nnz/n))), 2, 64) lanes).
// out[0..3] = format, algorithm, lanes, stages run; out[4..6] = the raw
// stage classes (-1 if not run); out[7] = configuration id.
__device__ void cascade(const DevModel &m, const double *f, int64_t n, int64_t nnz,
                        int32_t *out) {
    const int64_t mean = n > 0 ? nnz / n : 0;
    int lanes = 1;
    while ((int64_t)lanes * 2 <= mean && lanes < 64)
        lanes *= 2;
    if (lanes < 2)
        lanes = 2;
    int fmt = walk(m.t[0], f), alg = -1, lg = -1, stages = 1;
    int a = CK_ALG_VECTOR;
    if (fmt != CK_FMT_CSR) {
        a = 0;
        lanes = 0;
    } else {
        alg = walk(m.t[1], f);
        a = alg;
        stages = 2;
        if (alg != CK_ALG_VECTOR) {
            lanes = 0;
        } else {
            lg = walk(m.t[2], f);
            lanes = 1 << lg;
            stages = 3;
        }
    }
    out[0] = fmt;
    out[1] = a;
    out[2] = lanes;
    out[3] = stages;
    out[4] = fmt;
    out[5] = alg;
    out[6] = lg;
    out[7] = config_id_of(fmt, a, lanes);
}

__global__ void cascade_from_ints(DevModel m, const int64_t *I, int32_t *out) {
    if (threadIdx.x != 0 || blockIdx.x != 0)
        return;
    double d[9], f[kNumModelFeatures];
    derive_inputs(I, d);
    model_inputs_from(I, d, f);
    cascade(m, f, I[0], I[2], out);
}

// rows of 15 model inputs -> configuration ids
__global__ __launch_bounds__(256) void cascade_rows(DevModel m, int64_t count,
                                                    const double *__restrict__ f15,
                                                    int32_t *__restrict__ ids) {
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= count)
        return;
    double f[kNumModelFeatures];
    for (int k = 0; k < kNumModelFeatures; ++k)
        f[k] = f15[r * kNumModelFeatures + k];
    int32_t out[8];
    cascade(m, f, (int64_t)f[0], (int64_t)f[2], out);
    ids[r] = out[7];
}

// Node tables of the default model, uploaded once per device (kept until the
// process ends, like the model itself).
std::mutex g_dev_mu;
std::map<int, DevModel> g_dev_models;

ck_status device_model(DevModel &out) {
    int dev = 0;
    CK_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_dev_mu);
    auto it = g_dev_models.find(dev);
    if (it != g_dev_models.end()) {
        out = it->second;
        return CK_OK;
    }
    std::string err;
    const Cascade *C = load_cascade(nullptr, err);
    if (!C)
        return fail(CK_E_INVALID, "%s", err.c_str());
    DevModel m{};
    for (int t = 0; t < 3; ++t) {
        const Tree &T = C->tree[t];
        const size_t nn = T.feature.size();
        int *ints = nullptr;
        double *thr = nullptr;
        CK_HIP(hipMalloc((void **)&ints, 4 * nn * sizeof(int)));
        CK_HIP(hipMalloc((void **)&thr, nn * sizeof(double)));
        CK_HIP(hipMemcpy(ints, T.feature.data(), nn * sizeof(int), hipMemcpyHostToDevice));
        CK_HIP(hipMemcpy(ints + nn, T.left.data(), nn * sizeof(int), hipMemcpyHostToDevice));
        CK_HIP(hipMemcpy(ints + 2 * nn, T.right.data(), nn * sizeof(int), hipMemcpyHostToDevice));
        CK_HIP(hipMemcpy(ints + 3 * nn, T.cls.data(), nn * sizeof(int), hipMemcpyHostToDevice));
        CK_HIP(hipMemcpy(thr, T.threshold.data(), nn * sizeof(double), hipMemcpyHostToDevice));
        m.t[t] = DevTree{ints, ints + nn, ints + 2 * nn, ints + 3 * nn, thr};
    }
    g_dev_models[dev] = m;
    out = m;
    return CK_OK;
}

}  // namespace
}  // namespace ck

using namespace ck;

extern "C" {

ck_status ck_select_device(ck_handle h, int32_t *d_out, hipStream_t s) {
    if (!h || !d_out)
        return fail(CK_E_INVALID, "NULL argument");
    DevModel m;
    CK_TRY(device_model(m));   // the first call on a device uploads the trees (blocking)
    ck_matrix &M = *h;
    {
        std::lock_guard<std::mutex> lk(M.mu);
        if (!M.devsel_scratch) {
            // feature scratch + the 28 integers, kept with the handle so that
            // the call stays stream-ordered (nothing is given back while the
            // kernels may still run)
            const int64_t bytes = features_scratch_bytes(M.n, M.ncols, M.nnz) + 28 * 8 + 256;
            CK_TRY(mat_alloc(M, &M.devsel_scratch, bytes, s));
            M.devsel_ints = (int64_t *)(M.devsel_scratch +
                                        ((features_scratch_bytes(M.n, M.ncols, M.nnz) + 255) / 256) * 256);
        }
    }
    CK_TRY(launch_features(M, M.devsel_scratch, false, s));
    CK_TRY(launch_feature_ints(M, M.devsel_scratch, false, M.devsel_ints, s));
    hipLaunchKernelGGL(cascade_from_ints, dim3(1), dim3(64), 0, s, m, M.devsel_ints, d_out);
    CK_HIP(hipGetLastError());
    return CK_OK;
}

ck_status ck_cascade_eval_device(const double *d_f15, int64_t count, int32_t *d_ids,
                                 hipStream_t s) {
    if (count < 0 || (count > 0 && (!d_f15 || !d_ids)))
        return fail(CK_E_INVALID, "bad arguments");
    DevModel m;
    CK_TRY(device_model(m));
    if (count == 0)
        return CK_OK;
    hipLaunchKernelGGL(cascade_rows, dim3(ceil_div(count, 256)), dim3(256), 0, s, m, count, d_f15,
                       d_ids);
    CK_HIP(hipGetLastError());
    return CK_OK;
}

}  // extern "C"
