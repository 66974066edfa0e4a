// CSR-panel SpMV (XCD-aware column panels), see panel.hip.  G_dot = dot
// partials for a fused CG step.
#pragma once

#include "matrix.hpp"

namespace ck {

// panels for a vector of ncols entries of value_bytes each (x slice <= 2 MB)
int panel_count_for(int64_t ncols, int value_bytes);
int64_t panel_scan_tmp_elems(int64_t N);
// The panel count of M's CSR-panel copy: panel_count_for(ncols, 8), or 4
// (see panel.hip).  tmp: scratch of at least panel_count_for(ncols, 8) * n
// + 2 ints; returns when decided.  *counted: tmp[0 .. P n) already holds the
// chosen P's per-row panel counts (true when P = 4 was chosen).
ck_status panel_choose_count(const ck_matrix &M, int *tmp, hipStream_t s, int *P_out,
                             bool *counted);
// Exclusive scan of N ints into N + 1 outputs (out[N] = total); tmp holds
// panel_scan_tmp_elems(N) ints.
ck_status launch_scan_exclusive(int64_t N, const int *in, int *out, int *tmp, hipStream_t s);
ck_status launch_to_panel(const ck_matrix &M, int P, int64_t W, int *cnt, int *tmp, int *prp,
                          int *pcol, double *pval, float *pval32, bool counted, hipStream_t s);
// After launch_to_panel (cnt = its per-panel-row counts, M.panel_rp the
// dense row pointers): switch M to the row-list layout when at most 3/4 of
// the P*n panel rows are non-empty (cnt is overwritten).  Returns when done.
ck_status panel_make_rows(ck_matrix &M, int *cnt, hipStream_t s);
// y = alpha * (sum of the P partial vectors, in panel order) + beta * y
template <typename T>
ck_status launch_panel_combine(const ck_matrix &M, const SpmvArgs<T> &a, const T *ypart,
                               int64_t G_dot, hipStream_t s);

}  // namespace ck
