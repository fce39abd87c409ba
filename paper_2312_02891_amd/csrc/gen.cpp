// Host-side problem construction: the convection-diffusion matrices of Sec. 4
// (eq. (ex:convdiff)) in CSR form, upwind or central first differences, and
// a CSR transpose.
//
// This file must be compiled with -ffp-contract=off: every product and sum
// of the value recipe is rounded on its own, so the stored FP64 values are
// reproducible bit for bit.
#include <cmath>
#include <cstdint>
#include <algorithm>
#include <vector>

#include "../../include/lradi.h"

namespace lradi {
void set_error(const char* fmt, ...);
}

extern "C" int lradi_convdiff_size(int dim, int N, int64_t* n, int64_t* nnz) {
  if ((dim != 2 && dim != 3) || N < 1) {
    lradi::set_error("lradi_convdiff_size: dim must be 2 or 3 and N >= 1");
    return LRADI_EINVAL;
  }
  int64_t p = 1, q = 1;
  for (int c = 0; c < dim; ++c) p *= N;
  for (int c = 0; c < dim - 1; ++c) q *= N;
  if (p > INT32_MAX) {
    lradi::set_error("lradi_convdiff_size: N^dim exceeds int32 rows");
    return LRADI_EINVAL;
  }
  if (n) *n = p;
  if (nnz) *nnz = (2 * dim + 1) * p - 2 * dim * q;
  return LRADI_OK;
}

extern "C" int lradi_gen_convdiff_scheme(int dim, int N, const double* omega, int scheme,
                                         int32_t* rowptr, int32_t* colind, double* val) {
  int64_t n = 0, nnz = 0;
  int st = lradi_convdiff_size(dim, N, &n, &nnz);
  if (st != LRADI_OK) return st;
  if (!omega || !rowptr || !colind || !val) {
    lradi::set_error("lradi_gen_convdiff: null pointer");
    return LRADI_EINVAL;
  }
  if (scheme != LRADI_SCHEME_UPWIND && scheme != LRADI_SCHEME_CENTRAL) {
    lradi::set_error("lradi_gen_convdiff: unknown scheme %d", scheme);
    return LRADI_EINVAL;
  }
  if (nnz > INT32_MAX) {
    lradi::set_error("lradi_gen_convdiff: nnz exceeds int32 indices");
    return LRADI_EINVAL;
  }
  // coefficients of L_h (positive diagonal); A = -L_h
  const double ih = (double)(N + 1);
  const double ih2 = ih * ih;
  double lo[3], hi[3];
  double diag = 0.0;
  for (int c = 0; c < dim; ++c) {
    const double w = omega[c];
    const double twoih2 = 2.0 * ih2;
    if (scheme == LRADI_SCHEME_CENTRAL) {
      // central first difference: w_c (u_{p+s} - u_{p-s}) / (2h)
      const double half = (w * ih) * 0.5;
      lo[c] = -ih2 - half;
      hi[c] = -ih2 + half;
      diag = diag + twoih2;
      continue;
    }
    const double wp = w > 0.0 ? w : 0.0;
    const double wm = (-w) > 0.0 ? (-w) : 0.0;
    const double tlo = wp * ih;
    const double thi = wm * ih;
    lo[c] = -ih2 - tlo;  // neighbour p - s_c
    hi[c] = -ih2 - thi;  // neighbour p + s_c
    const double aw = std::fabs(w) * ih;
    const double term = twoih2 + aw;
    diag = diag + term;
  }
  int64_t stride[3] = {1, N, (int64_t)N * N};
  int64_t k = 0;
  rowptr[0] = 0;
  for (int64_t p = 0; p < n; ++p) {
    int64_t coord[3];
    for (int c = 0; c < dim; ++c) coord[c] = (p / stride[c]) % N;
    // ascending columns: p - s_{d-1}, ..., p - s_0, p, p + s_0, ..., p + s_{d-1}
    for (int c = dim - 1; c >= 0; --c) {
      if (coord[c] > 0) {
        colind[k] = (int32_t)(p - stride[c]);
        val[k] = -lo[c];
        ++k;
      }
    }
    colind[k] = (int32_t)p;
    val[k] = -diag;
    ++k;
    for (int c = 0; c < dim; ++c) {
      if (coord[c] < N - 1) {
        colind[k] = (int32_t)(p + stride[c]);
        val[k] = -hi[c];
        ++k;
      }
    }
    rowptr[p + 1] = (int32_t)k;
  }
  return (k == nnz) ? LRADI_OK : LRADI_EINVAL;
}

extern "C" int lradi_gen_convdiff(int dim, int N, const double* omega, int32_t* rowptr,
                                  int32_t* colind, double* val) {
  return lradi_gen_convdiff_scheme(dim, N, omega, LRADI_SCHEME_UPWIND, rowptr, colind, val);
}

namespace lradi {

// Transpose of an n x n CSR matrix (host arrays), columns ascending.
void csr_transpose(int n, const int32_t* rp, const int32_t* ci, const double* v,
                   std::vector<int32_t>& trp, std::vector<int32_t>& tci, std::vector<double>& tv) {
  const int64_t nnz = rp[n];
  trp.assign(n + 1, 0);
  tci.resize(nnz);
  tv.resize(nnz);
  for (int64_t k = 0; k < nnz; ++k) trp[ci[k] + 1] += 1;
  for (int i = 0; i < n; ++i) trp[i + 1] += trp[i];
  std::vector<int64_t> pos(trp.begin(), trp.end() - 1);
  for (int i = 0; i < n; ++i)
    for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
      const int64_t dst = pos[ci[k]]++;
      tci[dst] = i;
      tv[dst] = v[k];
    }
}

// Union pattern of two n x n CSR matrices P and Q (columns ascending per
// row; duplicate entries within one matrix are summed) with both value
// arrays on it: the pencil P + s Q is stored once, its values formed per
// shift on the device.
void csr_union(int n, const int32_t* prp, const int32_t* pci, const double* pv, const int32_t* qrp,
               const int32_t* qci, const double* qv, std::vector<int32_t>& urp,
               std::vector<int32_t>& uci, std::vector<double>& upv, std::vector<double>& uqv) {
  urp.assign(n + 1, 0);
  uci.clear();
  upv.clear();
  uqv.clear();
  std::vector<std::pair<int32_t, int>> row;  // (column, which) sorted
  std::vector<double> vals;
  for (int i = 0; i < n; ++i) {
    row.clear();
    for (int64_t k = prp[i]; k < prp[i + 1]; ++k) row.push_back({pci[k], (int)(k - prp[i])});
    const int np = (int)row.size();
    for (int64_t k = qrp[i]; k < qrp[i + 1]; ++k) row.push_back({qci[k], np + (int)(k - qrp[i])});
    std::stable_sort(row.begin(), row.end(),
                     [](const std::pair<int32_t, int>& a, const std::pair<int32_t, int>& b) {
                       return a.first < b.first;
                     });
    for (size_t e = 0; e < row.size(); ++e) {
      const int32_t col = row[e].first;
      const int src = row[e].second;
      const double pvv = src < np ? pv[prp[i] + src] : 0.0;
      const double qvv = src < np ? 0.0 : qv[qrp[i] + (src - np)];
      if (!uci.empty() && (int64_t)uci.size() > urp[i] && uci.back() == col) {
        upv.back() += pvv;
        uqv.back() += qvv;
      } else {
        uci.push_back(col);
        upv.push_back(pvv);
        uqv.push_back(qvv);
      }
    }
    urp[i + 1] = (int32_t)uci.size();
  }
}

}  // namespace lradi
