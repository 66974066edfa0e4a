// C-ABI entry points for the matrix store, features, prediction, conversion
// and SpMV (declared in include/caskrylov.h).
#include <algorithm>
#include <cstdarg>
#include <cstring>
#include <limits>

#include "matrix.hpp"
#include "devcache.hpp"
#include "diahyb.hpp"
#include "panel.hpp"
#include "predictor.hpp"
#include "solvers.hpp"

namespace ck {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

ck_status fail(ck_status st, const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

// features.hip
ck_status launch_validate(int64_t n, int64_t ncols, int64_t nnz, const int *rp, const int *col,
                          unsigned *state, hipStream_t s);
int64_t validate_state_elems(int64_t nnz);
int64_t features_scratch_bytes(int64_t n, int64_t ncols, int64_t nnz);
ck_status launch_features(const ck_matrix &M, void *scratch, bool symmetry, hipStream_t s);
void features_from_acc(const void *acc_host, const ck_matrix &M, int64_t *out28);
int64_t features_acc_offset(int64_t n, int64_t ncols);
size_t features_acc_size();
ck_status launch_row_max(int64_t n, const int *rp, unsigned long long *out, hipStream_t s);
ck_status launch_to_ell(const ck_matrix &M, int64_t K, int64_t pitch, int *ecol, double *evl,
                        float *evl32, hipStream_t s);
ck_status launch_to_coo(const ck_matrix &M, int *row, hipStream_t s);

static void release(ck_matrix *M) {
    if (!M)
        return;
    mat_free(*M, M->rp);
    mat_free(*M, M->col);
    mat_free(*M, M->val);
    mat_free(*M, M->val32);
    mat_free(*M, M->ell_col);
    mat_free(*M, M->ell_val);
    mat_free(*M, M->ell_val32);
    mat_free(*M, M->coo_row);
    mat_free(*M, M->dia_off);
    mat_free(*M, M->dia_val);
    mat_free(*M, M->dia_val32);
    mat_free(*M, M->hyb_col);
    mat_free(*M, M->hyb_val);
    mat_free(*M, M->hyb_val32);
    mat_free(*M, M->hyb_rows);
    mat_free(*M, M->panel_rp);
    mat_free(*M, M->panel_col);
    mat_free(*M, M->panel_val);
    mat_free(*M, M->panel_val32);
    mat_free(*M, M->merge_part);
    mat_free(*M, M->panel_part);
    mat_free(*M, M->panel_row);
    mat_free(*M, M->devsel_scratch);
    mat_free(*M, M->panel_boff);
    for (auto &kv : M->carry)
        mat_free(*M, kv.second);
    delete M;
}

// Exact integer features (GPU) plus host-derived floating-point features.
// `symmetry` = false skips the transposed-entry search (is_symmetric is then
// reported as 0): the cascade does not use it, so a solve's own feature pass
// leaves it out.
ck_status compute_features(ck_matrix &M, ck_features &F, hipStream_t s, bool symmetry) {
    std::memset(&F, 0, sizeof F);
    const int64_t bytes = features_scratch_bytes(M.n, M.ncols, M.nnz);
    char *scratch = nullptr;
    CK_TRY(mat_alloc(M, &scratch, bytes, s));
    ck_status st = launch_features(M, scratch, symmetry, s);
    char acc[512];
    if (st == CK_OK) {
        const hipError_t e = hipMemcpyAsync(acc, (char *)scratch + features_acc_offset(M.n, M.ncols),
                                            features_acc_size(), hipMemcpyDeviceToHost, s);
        if (e != hipSuccess)
            st = fail(CK_E_HIP, "feature copy failed: %s", hipGetErrorString(e));
    }
    const hipError_t es = hipStreamSynchronize(s);
    mat_free(M, scratch);   // the pass has finished with it
    CK_TRY(st);
    if (es != hipSuccess)
        return fail(CK_E_HIP, "feature pass failed: %s", hipGetErrorString(es));
    int64_t ints[28];
    features_from_acc(acc, M, ints);
    if (!symmetry)
        ints[27] = 0;
    std::memcpy(&F, ints, sizeof ints);
    derive_features(F);
    M.max_row = F.max_r;
    return CK_OK;
}

// A format copy is marked available only once every kernel that builds it
// has finished: other threads use it at once on other streams (the request
// loop's workers, a solve given the configuration), and a flag set at
// enqueue time let them read half-built index arrays.
static ck_status mark_built(std::atomic<bool> &flag, hipStream_t s) {
    CK_HIP(hipStreamSynchronize(s));
    flag.store(true);
    return CK_OK;
}

// Builds the ELL, COO, DIA, HYB or CSR-panel copy (or the merge-path
// partition) a configuration needs (idempotent); returns when it is built.
ck_status convert_format(ck_matrix &M, const ck_config &c, hipStream_t s) {
    if (!config_valid(c))
        return fail(CK_E_INVALID, "invalid SpMV configuration");
    if (c.format == CK_FMT_CSR && c.algorithm != CK_ALG_PANEL && c.algorithm != CK_ALG_MERGE)
        return CK_OK;
    std::lock_guard<std::mutex> lk(M.mu);
    if (c.format == CK_FMT_CSR && c.algorithm == CK_ALG_MERGE) {
        // the merge-path partition of the matrix, searched once instead of by
        // every workgroup of every product
        if (M.has_merge_part.load())
            return CK_OK;
        CK_TRY(mat_alloc(M, &M.merge_part, merge_part_entries(M), s));
        CK_TRY(launch_merge_partition(M, M.merge_part, s));
        return mark_built(M.has_merge_part, s);
    }
    if (c.format == CK_FMT_CSR) {   // CSR-panel
        if (M.has_panel.load())
            return CK_OK;
        const int P8 = panel_count_for(M.ncols, 8);
        const int64_t N8 = (int64_t)P8 * M.n;   // the most panel rows P can give
        if (N8 + 1 > (int64_t)std::numeric_limits<int32_t>::max())
            return fail(CK_E_UNSUPPORTED, "too many panel rows");
        int *tmp = nullptr;
        CK_TRY(mat_alloc(M, &tmp, N8 + 2 + panel_scan_tmp_elems(N8), s));
        int P = P8;
        bool counted = false;
        ck_status st = panel_choose_count(M, tmp, s, &P, &counted);
        const int64_t W = ceil_div(std::max<int64_t>(M.ncols, 1), P);
        const int64_t N = (int64_t)P * M.n;
        if (st == CK_OK)
            st = mat_alloc(M, &M.panel_rp, N + 1, s);
        if (st == CK_OK)
            st = mat_alloc(M, &M.panel_col, M.nnz, s);
        if (st == CK_OK)
            st = mat_alloc(M, &M.panel_val, M.nnz, s);
        if (st == CK_OK && M.val32)
            st = mat_alloc(M, &M.panel_val32, M.nnz, s);
        if (st == CK_OK)
            st = launch_to_panel(M, P, W, tmp, tmp + N, M.panel_rp, M.panel_col, M.panel_val,
                                 M.panel_val32, counted, s);
        M.panel_P = P;
        M.panel_W = W;
        M.panel_rows = N;
        if (st == CK_OK)
            st = panel_make_rows(M, tmp, s);   // only the non-empty panel rows, if that pays
        const int64_t R = M.panel_rows;
        if (st == CK_OK)
            st = mat_alloc(M, &M.panel_part, merge_part_entries_rows(R, M.nnz), s);
        if (st == CK_OK)
            st = launch_merge_partition_rows(R, M.nnz, M.panel_rp, M.panel_part, s);
        if (st == CK_OK)
            st = mark_built(M.has_panel, s);
        (void)hipStreamSynchronize(s);   // the conversion has finished with tmp
        mat_free(M, tmp);
        return st;
    }
    if (c.format == CK_FMT_DIA) {
        if (M.has_dia.load())
            return CK_OK;
        const ck_status st = convert_to_dia(M, s);
        if (st != CK_OK) {   // refused for fill, or out of memory: leave no partial copy
            (void)hipStreamSynchronize(s);
            mat_free(M, M.dia_off);
            mat_free(M, M.dia_val);
            mat_free(M, M.dia_val32);
            M.dia_off = nullptr;
            M.dia_val = nullptr;
            M.dia_val32 = nullptr;
            return st;
        }
        return mark_built(M.has_dia, s);
    }
    if (c.format == CK_FMT_HYB) {
        if (M.has_hyb.load())
            return CK_OK;
        const ck_status st = convert_to_hyb(M, s);
        if (st != CK_OK) {
            (void)hipStreamSynchronize(s);
            mat_free(M, M.hyb_col);
            mat_free(M, M.hyb_val);
            mat_free(M, M.hyb_val32);
            mat_free(M, M.hyb_rows);
            M.hyb_col = nullptr;
            M.hyb_val = nullptr;
            M.hyb_val32 = nullptr;
            M.hyb_rows = nullptr;
            return st;
        }
        return mark_built(M.has_hyb, s);
    }
    if (c.format == CK_FMT_COO) {
        if (M.has_coo.load())
            return CK_OK;
        CK_TRY(mat_alloc(M, &M.coo_row, M.nnz, s));
        CK_TRY(launch_to_coo(M, M.coo_row, s));
        return mark_built(M.has_coo, s);
    }
    if (M.has_ell.load())
        return CK_OK;
    if (M.max_row < 0) {
        unsigned long long *d = nullptr;
        unsigned long long h = 0;
        CK_TRY(mat_alloc(M, &d, 1, s));
        ck_status st = launch_fill<int>(2, (int *)d, 0, s);
        if (st == CK_OK)
            st = launch_row_max(M.n, M.rp, d, s);
        if (st == CK_OK && hipMemcpyAsync(&h, d, sizeof h, hipMemcpyDeviceToHost, s) != hipSuccess)
            st = fail(CK_E_HIP, "row-length read-back failed");
        if (hipStreamSynchronize(s) != hipSuccess && st == CK_OK)
            st = fail(CK_E_HIP, "row-length pass failed");
        mat_free(M, d);
        CK_TRY(st);
        M.max_row = (int64_t)h;
    }
    const int64_t K = M.max_row;
    const int64_t pitch = ceil_div(M.n, 64) * 64;
    if (K * pitch > 8 * M.nnz)
        return fail(CK_E_UNSUPPORTED, "ELL refused: %lld slots for %lld stored entries",
                    (long long)(K * pitch), (long long)M.nnz);
    CK_TRY(mat_alloc(M, &M.ell_col, K * pitch, s));
    CK_TRY(mat_alloc(M, &M.ell_val, K * pitch, s));
    if (M.val32)
        CK_TRY(mat_alloc(M, &M.ell_val32, K * pitch, s));
    CK_TRY(launch_to_ell(M, K, pitch, M.ell_col, M.ell_val, M.ell_val32, s));
    M.ell_K = K;
    M.ell_pitch = pitch;
    return mark_built(M.has_ell, s);
}

}  // namespace ck

using namespace ck;

extern "C" {

const char *ck_last_error(void) { return g_last_error.c_str(); }

int32_t ck_config_id(const ck_config *c) {
    if (!c || !config_valid(*c))
        return -1;
    if (c->format == CK_FMT_ELL)
        return 9;
    if (c->format == CK_FMT_COO)
        return 10;
    if (c->format == CK_FMT_DIA)
        return 12;
    if (c->format == CK_FMT_HYB)
        return 13;
    if (c->algorithm == CK_ALG_SCALAR)
        return 7;
    if (c->algorithm == CK_ALG_MERGE)
        return 8;
    if (c->algorithm == CK_ALG_PANEL)
        return 11;
    int idx = 0;
    while ((1 << idx) < c->lanes)
        ++idx;
    return idx;
}

ck_status ck_config_from_id(int32_t id, ck_config *out) {
    if (!out || id < 0 || id >= CK_NUM_CONFIGS)
        return fail(CK_E_INVALID, "configuration id must be in [0, %d]", CK_NUM_CONFIGS - 1);
    if (id == 11) {
        *out = ck_config{CK_FMT_CSR, CK_ALG_PANEL, 0, 0};
        return CK_OK;
    }
    if (id == 12 || id == 13) {
        *out = ck_config{id == 12 ? CK_FMT_DIA : CK_FMT_HYB, 0, 0, 0};
        return CK_OK;
    }
    if (id <= 6)
        *out = ck_config{CK_FMT_CSR, CK_ALG_VECTOR, 1 << id, 0};
    else if (id == 7)
        *out = ck_config{CK_FMT_CSR, CK_ALG_SCALAR, 0, 0};
    else if (id == 8)
        *out = ck_config{CK_FMT_CSR, CK_ALG_MERGE, 0, 0};
    else if (id == 9)
        *out = ck_config{CK_FMT_ELL, 0, 0, 0};
    else
        *out = ck_config{CK_FMT_COO, 0, 0, 0};
    return CK_OK;
}

ck_status ck_kernel_name(const ck_config *cfg, int32_t fp32, char *buf, size_t cap) {
    if (!cfg || !buf || cap == 0 || !config_valid(*cfg))
        return fail(CK_E_INVALID, "bad arguments");
    snprintf(buf, cap, "%s", kernel_name(*cfg, fp32 != 0));
    return CK_OK;
}

ck_status spmv_create(ck_handle *out, int64_t nrows, int64_t ncols, int64_t nnz,
                      const int32_t *d_rowptr, const int32_t *d_col, const double *d_val,
                      uint32_t flags, const ck_allocator *alloc, hipStream_t s) {
    if (!out)
        return fail(CK_E_INVALID, "out is NULL");
    *out = nullptr;
    const int64_t lim = std::numeric_limits<int32_t>::max() - 4096;
    if (nrows < 0 || ncols < 0 || nnz < 0 || nrows > lim || ncols > lim || nnz > lim)
        return fail(CK_E_INVALID, "sizes must be non-negative and fit int32 indexing");
    if (!d_rowptr || (nnz > 0 && (!d_col || !d_val)))
        return fail(CK_E_INVALID, "NULL CSR array");
    if (flags & ~CK_KEEP_FP32)
        return fail(CK_E_INVALID, "unknown flags");
    if (alloc && (!alloc->alloc || !alloc->free))
        return fail(CK_E_INVALID, "allocator without alloc or free function");
    ck_matrix *M = new ck_matrix();
    if (alloc) {
        M->mem.a = *alloc;
        M->mem.user = true;
    }
    M->n = nrows;
    M->ncols = ncols;
    M->nnz = nnz;
    M->flags = flags;
    (void)hipGetDevice(&M->device);
    ck_status st = CK_OK;
    unsigned *bad = nullptr;
    unsigned hbad = 0;
    do {
        if ((st = mat_alloc(*M, &M->rp, nrows + 1, s)) != CK_OK) break;
        if ((st = mat_alloc(*M, &M->col, nnz, s)) != CK_OK) break;
        if ((st = mat_alloc(*M, &M->val, nnz, s)) != CK_OK) break;
        hipError_t e = hipMemcpyAsync(M->rp, d_rowptr, sizeof(int32_t) * (nrows + 1),
                                      hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess && nnz > 0)
            e = hipMemcpyAsync(M->col, d_col, sizeof(int32_t) * nnz, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess && nnz > 0)
            e = hipMemcpyAsync(M->val, d_val, sizeof(double) * nnz, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) {
            st = fail(CK_E_HIP, "copy of the CSR arrays failed: %s", hipGetErrorString(e));
            break;
        }
        if (flags & CK_KEEP_FP32) {
            if ((st = mat_alloc(*M, &M->val32, nnz, s)) != CK_OK) break;
            if (nnz > 0 && (st = launch_copy<float, double>(nnz, M->val32, M->val, nullptr, s)) != CK_OK)
                break;
        }
        if ((st = mat_alloc(*M, &bad, validate_state_elems(nnz), s)) != CK_OK) break;
        if ((st = launch_fill<int>(2, (int *)bad, 0, s)) != CK_OK) break;
        if ((st = launch_validate(nrows, ncols, nnz, M->rp, M->col, bad, s)) != CK_OK) break;
        e = hipMemcpyAsync(&hbad, bad, sizeof hbad, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            st = fail(CK_E_HIP, "validation failed: %s", hipGetErrorString(e));
            break;
        }
        if (hbad) {
            st = fail(CK_E_INVALID, "malformed CSR (code %u): rowptr must start at 0, be "
                      "nondecreasing and end at nnz; columns in range and strictly increasing",
                      hbad);
            break;
        }
    } while (false);
    (void)hipStreamSynchronize(s);   // nothing may still write the arrays
    mat_free(*M, bad);
    if (st != CK_OK) {
        release(M);
        return st;
    }
    M->active = default_config(nrows, nnz);
    *out = M;
    return CK_OK;
}

void spmv_destroy(ck_handle h) { release(h); }

ck_status spmv_features(ck_handle h, ck_features *out, hipStream_t s) {
    if (!h || !out)
        return fail(CK_E_INVALID, "NULL argument");
    return compute_features(*h, *out, s, true);
}

ck_status ck_features_ex(ck_handle h, ck_features *out, uint32_t flags, hipStream_t s) {
    if (!h || !out)
        return fail(CK_E_INVALID, "NULL argument");
    if (flags & ~CK_FEAT_NO_SYMMETRY)
        return fail(CK_E_INVALID, "unknown feature flags 0x%x", flags);
    const bool symmetry = !(flags & CK_FEAT_NO_SYMMETRY);
    CK_TRY(compute_features(*h, *out, s, symmetry));
    if (!symmetry)
        out->is_symmetric = -1;
    return CK_OK;
}

ck_status ck_select_stages(const ck_features *f, const char *model_path, int32_t stage[3]) {
    if (!f || !stage)
        return fail(CK_E_INVALID, "NULL argument");
    std::string err;
    const Cascade *C = load_cascade(model_path, err);
    if (!C)
        return fail(CK_E_INVALID, "%s", err.c_str());
    double in[kNumModelFeatures];
    model_inputs(*f, in);
    stage[0] = C->tree[0].eval(in);
    stage[1] = -1;
    stage[2] = -1;
    if (stage[0] == CK_FMT_CSR) {
        stage[1] = C->tree[1].eval(in);
        if (stage[1] == CK_ALG_VECTOR)
            stage[2] = C->tree[2].eval(in);
    }
    if (stage[0] < 0 || stage[0] > CK_FMT_HYB || stage[1] > CK_ALG_PANEL || stage[2] > 6)
        return fail(CK_E_INVALID, "cascade model produced an unknown class");
    return CK_OK;
}

ck_status ck_eval_stage(const ck_features *f, const char *model_path, int32_t stage,
                        int32_t *cls) {
    if (!f || !cls || stage < 0 || stage > 2)
        return fail(CK_E_INVALID, "bad arguments");
    std::string err;
    const Cascade *C = load_cascade(model_path, err);
    if (!C)
        return fail(CK_E_INVALID, "%s", err.c_str());
    double in[kNumModelFeatures];
    model_inputs(*f, in);
    *cls = C->tree[stage].eval(in);
    return CK_OK;
}

ck_status spmv_select(const ck_features *f, const char *model_path, ck_config *out) {
    if (!f || !out)
        return fail(CK_E_INVALID, "NULL argument");
    int32_t st[3];
    CK_TRY(ck_select_stages(f, model_path, st));
    ck_config c = default_config(f->nrows, f->nnz);
    for (int t = 0; t < 3 && st[t] >= 0; ++t)
        c = stage_config(t, st[t], c);
    *out = c;
    return CK_OK;
}

ck_status ck_start_config(int64_t nrows, int64_t ncols, int64_t nnz, const char *model_path,
                          ck_config *out, int32_t *from_tree) {
    if (!out)
        return fail(CK_E_INVALID, "NULL argument");
    if (nrows < 0 || ncols < 0 || nnz < 0)
        return fail(CK_E_INVALID, "negative dimension");
    std::string err;
    const Cascade *C = load_cascade(model_path, err);
    if (!C)
        return fail(CK_E_INVALID, "%s", err.c_str());
    *out = default_config(nrows, nnz);
    if (from_tree)
        *from_tree = 0;
    const int id = nrows > 0 ? start_config_id(*C, nrows, ncols, nnz) : -1;
    if (id >= 0) {
        CK_TRY(ck_config_from_id(id, out));
        if (from_tree)
            *from_tree = 1;
    }
    return CK_OK;
}

ck_status ck_default_config(ck_handle h, ck_config *out) {
    if (!h || !out)
        return fail(CK_E_INVALID, "NULL argument");
    *out = default_config(h->n, h->nnz);
    return CK_OK;
}

ck_status spmv_convert(ck_handle h, const ck_config *cfg, hipStream_t s) {
    if (!h || !cfg)
        return fail(CK_E_INVALID, "NULL argument");
    return convert_format(*h, *cfg, s);
}

ck_status ck_set_active(ck_handle h, const ck_config *cfg) {
    if (!h || !cfg || !config_valid(*cfg))
        return fail(CK_E_INVALID, "bad configuration");
    if ((cfg->format == CK_FMT_ELL && !h->has_ell.load()) ||
        (cfg->format == CK_FMT_COO && !h->has_coo.load()) ||
        (cfg->format == CK_FMT_DIA && !h->has_dia.load()) ||
        (cfg->format == CK_FMT_HYB && !h->has_hyb.load()))
        return fail(CK_E_INVALID, "format not converted yet");
    std::lock_guard<std::mutex> lk(h->mu);
    h->active = *cfg;
    return CK_OK;
}

ck_status ck_get_active(ck_handle h, ck_config *out) {
    if (!h || !out)
        return fail(CK_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(h->mu);
    *out = h->active;
    return CK_OK;
}

static ck_config active_of(ck_handle h) {
    std::lock_guard<std::mutex> lk(h->mu);
    return h->active;
}

// Carry workspace for merge-path / COO products on stream s, sized for both.
static ck_status carry_for(ck_handle h, const ck_config &c, hipStream_t s, void **out) {
    *out = nullptr;
    if (!(c.format == CK_FMT_COO ||
          (c.format == CK_FMT_CSR && (c.algorithm == CK_ALG_MERGE || c.algorithm == CK_ALG_PANEL))))
        return CK_OK;
    std::lock_guard<std::mutex> lk(h->mu);
    auto it = h->carry.find(s);
    if (it != h->carry.end()) {
        *out = it->second;
        return CK_OK;
    }
    const int64_t bytes =
        std::max(spmv_carry_bytes(*h, ck_config{CK_FMT_CSR, CK_ALG_MERGE, 0, 0}, false),
                 std::max(spmv_carry_bytes(*h, ck_config{CK_FMT_COO, 0, 0, 0}, false),
                          spmv_carry_bytes(*h, ck_config{CK_FMT_CSR, CK_ALG_PANEL, 0, 0}, false)));
    char *p = nullptr;
    CK_TRY(mat_alloc(*h, &p, bytes, s));
    h->carry[s] = p;
    *out = p;
    return CK_OK;
}

ck_status spmv_apply(ck_handle h, const ck_config *cfg, double alpha, const double *d_x,
                     double beta, double *d_y, hipStream_t s) {
    if (!h || (h->n > 0 && !d_y) || (h->ncols > 0 && !d_x))
        return fail(CK_E_INVALID, "NULL argument");
    SpmvArgs<double> a;
    a.alpha = alpha;
    a.beta = beta;
    a.x = d_x;
    a.y = d_y;
    const ck_config c = cfg ? *cfg : active_of(h);
    CK_TRY(carry_for(h, c, s, &a.carry));
    return launch_spmv<double>(*h, c, a, s);
}

// ---- allocation-free product ------------------------------------------------
// The carry workspace of spmv_apply_noalloc (merge-path and COO carries,
// CSR-panel partial vectors) lives in this fixed device array, one copy per
// GPU for the life of the process.  In host code `scratch` only names the
// symbol; its device address on the current GPU comes from
// hipGetSymbolAddress, looked up once per device and kept.
constexpr int64_t kNoAllocScratchBytes = int64_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

static std::mutex g_scratch_mu;
static std::map<int, void *> g_scratch_ptr;   // device -> address of its `scratch`

static ck_status scratch_ptr(void **out) {
    int dev = 0;
    CK_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it == g_scratch_ptr.end()) {
        void *p = nullptr;
        CK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p)
            return fail(CK_E_HIP, "no device address for the scratch array on device %d", dev);
        it = g_scratch_ptr.emplace(dev, p).first;
    }
    *out = it->second;
    return CK_OK;
}

ck_status spmv_apply_noalloc(ck_handle h, const ck_config *cfg, double alpha, const double *d_x,
                             double beta, double *d_y, hipStream_t s) {
    if (!h || (h->n > 0 && !d_y) || (h->ncols > 0 && !d_x))
        return fail(CK_E_INVALID, "NULL argument");
    SpmvArgs<double> a;
    a.alpha = alpha;
    a.beta = beta;
    a.x = d_x;
    a.y = d_y;
    const ck_config c = cfg ? *cfg : active_of(h);
    if (!config_valid(c))
        return fail(CK_E_INVALID, "invalid SpMV configuration");
    const bool carries = c.format == CK_FMT_COO ||
                         (c.format == CK_FMT_CSR &&
                          (c.algorithm == CK_ALG_MERGE || c.algorithm == CK_ALG_PANEL));
    if (carries && h->n > 0) {
        const int64_t need = spmv_carry_bytes(*h, c, false);
        if (need > kNoAllocScratchBytes)
            return fail(CK_E_UNSUPPORTED,
                        "spmv_apply_noalloc: %s needs %lld bytes of workspace for this matrix, "
                        "above the fixed %lld-byte scratch array (use spmv_apply)",
                        kernel_name(c, false), (long long)need, (long long)kNoAllocScratchBytes);
        CK_TRY(scratch_ptr(&a.carry));
    }
    return launch_spmv<double>(*h, c, a, s);
}

ck_status spmv_apply_f32(ck_handle h, const ck_config *cfg, float alpha, const float *d_x,
                         float beta, float *d_y, hipStream_t s) {
    if (!h || (h->n > 0 && !d_y) || (h->ncols > 0 && !d_x))
        return fail(CK_E_INVALID, "NULL argument");
    SpmvArgs<float> a;
    a.alpha = alpha;
    a.beta = beta;
    a.x = d_x;
    a.y = d_y;
    const ck_config c = cfg ? *cfg : active_of(h);
    CK_TRY(carry_for(h, c, s, &a.carry));
    return launch_spmv<float>(*h, c, a, s);
}

ck_status ck_export_ell(ck_handle h, int32_t *d_col, double *d_val, int64_t *K, int64_t *pitch,
                        hipStream_t s) {
    if (!h || !K || !pitch)
        return fail(CK_E_INVALID, "NULL argument");
    if (!h->has_ell.load())
        return fail(CK_E_INVALID, "matrix has no ELL copy");
    *K = h->ell_K;
    *pitch = h->ell_pitch;
    const size_t cnt = (size_t)(h->ell_K * h->ell_pitch);
    if (d_col && cnt)
        CK_HIP(hipMemcpyAsync(d_col, h->ell_col, cnt * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    if (d_val && cnt)
        CK_HIP(hipMemcpyAsync(d_val, h->ell_val, cnt * sizeof(double), hipMemcpyDeviceToDevice, s));
    return CK_OK;
}

ck_status ck_export_dia(ck_handle h, int32_t *d_off, double *d_val, int64_t *ndiag,
                        int64_t *pitch, hipStream_t s) {
    if (!h || !ndiag || !pitch)
        return fail(CK_E_INVALID, "NULL argument");
    if (!h->has_dia.load())
        return fail(CK_E_INVALID, "matrix has no DIA copy");
    *ndiag = h->dia_nd;
    *pitch = h->dia_pitch;
    if (d_off && h->dia_nd > 0)
        CK_HIP(hipMemcpyAsync(d_off, h->dia_off, h->dia_nd * sizeof(int32_t),
                              hipMemcpyDeviceToDevice, s));
    if (d_val && h->dia_nd > 0)
        CK_HIP(hipMemcpyAsync(d_val, h->dia_val, h->dia_nd * h->dia_pitch * sizeof(double),
                              hipMemcpyDeviceToDevice, s));
    return CK_OK;
}

ck_status ck_export_hyb(ck_handle h, int32_t *d_col, double *d_val, int32_t *d_rows, int64_t *K,
                        int64_t *pitch, int64_t *ntail, int32_t *lanes, hipStream_t s) {
    if (!h || !K || !pitch || !ntail || !lanes)
        return fail(CK_E_INVALID, "NULL argument");
    if (!h->has_hyb.load())
        return fail(CK_E_INVALID, "matrix has no HYB copy");
    *K = h->hyb_K;
    *pitch = h->hyb_pitch;
    *ntail = h->hyb_nt;
    *lanes = h->hyb_L;
    const size_t cnt = (size_t)(h->hyb_K * h->hyb_pitch);
    if (d_col && cnt)
        CK_HIP(hipMemcpyAsync(d_col, h->hyb_col, cnt * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    if (d_val && cnt)
        CK_HIP(hipMemcpyAsync(d_val, h->hyb_val, cnt * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (d_rows && h->hyb_nt > 0)
        CK_HIP(hipMemcpyAsync(d_rows, h->hyb_rows, h->hyb_nt * sizeof(int32_t),
                              hipMemcpyDeviceToDevice, s));
    return CK_OK;
}

ck_status ck_export_coo_rows(ck_handle h, int32_t *d_row, hipStream_t s) {
    if (!h || (!d_row && h->nnz > 0))
        return fail(CK_E_INVALID, "NULL argument");
    if (!h->has_coo.load())
        return fail(CK_E_INVALID, "matrix has no COO copy");
    if (h->nnz)
        CK_HIP(hipMemcpyAsync(d_row, h->coo_row, h->nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    return CK_OK;
}

ck_status ck_panel_layout(ck_handle h, int32_t *panels, int64_t *width, int64_t *stored_rows) {
    if (!h || !panels || !width || !stored_rows)
        return fail(CK_E_INVALID, "NULL argument");
    if (!h->has_panel.load())
        return fail(CK_E_INVALID, "matrix has no CSR-panel copy");
    *panels = h->panel_P;
    *width = h->panel_W;
    *stored_rows = h->panel_rows;
    return CK_OK;
}

ck_status ck_dot(int64_t n, const double *d_x, const double *d_y, double *d_out, hipStream_t s) {
    if (n < 0 || !d_out || (n > 0 && (!d_x || !d_y)))
        return fail(CK_E_INVALID, "bad arguments");
    void *ws = nullptr;
    CK_HIP(hipMallocAsync(&ws, 1024 * sizeof(double) + 256, s));
    const ck_status st = launch_dot(n, d_x, d_y, (double *)ws, d_out, s);
    CK_HIP(hipFreeAsync(ws, s));
    return st;
}

ck_status ck_time_spmv(ck_handle h, const ck_config *cfg, int32_t fp32, const void *d_x,
                       void *d_y, int32_t warmup, int32_t reps, hipStream_t s,
                       double *us_per_call) {
    if (!h || !cfg || !us_per_call || reps <= 0 || warmup < 0 ||
        (h->n > 0 && !d_y) || (h->ncols > 0 && !d_x))
        return fail(CK_E_INVALID, "bad arguments");
    void *carry = nullptr;
    CK_TRY(carry_for(h, *cfg, s, &carry));
    SpmvArgs<double> a64;
    SpmvArgs<float> a32;
    a64.x = (const double *)d_x;
    a64.y = (double *)d_y;
    a64.carry = carry;
    a32.x = (const float *)d_x;
    a32.y = (float *)d_y;
    a32.carry = carry;
    auto one = [&]() -> ck_status {
        return fp32 ? launch_spmv<float>(*h, *cfg, a32, s) : launch_spmv<double>(*h, *cfg, a64, s);
    };
    for (int i = 0; i < warmup; ++i)
        CK_TRY(one());
    hipEvent_t e0, e1;
    CK_HIP(hipEventCreate(&e0));
    CK_HIP(hipEventCreate(&e1));
    ck_status st = CK_OK;
    if (hipEventRecord(e0, s) != hipSuccess)
        st = fail(CK_E_HIP, "hipEventRecord failed");
    for (int i = 0; i < reps && st == CK_OK; ++i)
        st = one();
    float ms = 0.f;
    if (st == CK_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                        hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        st = fail(CK_E_HIP, "event timing failed");
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    CK_TRY(st);
    *us_per_call = 1000.0 * (double)ms / reps;
    return CK_OK;
}

int64_t ck_spmv_bytes(ck_handle h, int32_t fp32, int32_t beta_nonzero) {
    if (!h)
        return -1;
    const int64_t sz = fp32 ? 4 : 8;
    return h->nnz * (sz + 4) + 4 * (h->n + 1) + sz * h->ncols + sz * h->n +
           (beta_nonzero ? sz * h->n : 0);
}

}  // extern "C"
