// DIA and HYB formats: conversions and products (diahyb.hip).
#pragma once

#include "matrix.hpp"

namespace ck {

// Build M.dia_* (CK_E_UNSUPPORTED when ndiag * pitch > 8 * nnz) / M.hyb_*.
// Enqueued on s; both block on s once to read a count back.
ck_status convert_to_dia(ck_matrix &M, hipStream_t s);
ck_status convert_to_hyb(ck_matrix &M, hipStream_t s);

// DIA product over G logical row blocks (dot partials as the ELL kernel).
template <typename T, bool BETA, bool DOT>
void launch_dia_spmv(const ck_matrix &M, int64_t G, const T *dv, const SpmvArgs<T> &a,
                     hipStream_t s);
// HYB remainder pass: y[i] += alpha * (entries K.. of each long row i).
template <typename T>
void launch_hyb_tail(const ck_matrix &M, const T *val, const SpmvArgs<T> &a, hipStream_t s);

}  // namespace ck
