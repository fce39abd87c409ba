// The largest-eigenvalue routines of small.h with the bisection spread over
// L lanes of a wavefront (multisection): every lane of the group reduces
// the same matrix to tridiagonal form, tests its own point per round, and
// a ballot tells all of them the sub-interval to keep.  Each round gains
// log2(L + 1) bits for the latency of one Sturm count.  All lanes of a group
// call with the same matrix and get the same value.
#pragma once

#include <hip/hip_runtime.h>

#include "small.h"

namespace lradi {

// lane: 0..L-1 within the group; base: the group's first lane in the
// wavefront (a multiple of L)
template <int N, int L>
__device__ inline double lambda_max_sym_lanes_t(const double* G, int lane, int base) {
  LmaxTri<N> t;
  lmax_prepare<N>(G, t);
  if (t.done) return t.value;
  const unsigned long long gm = L == 64 ? ~0ull : ((1ull << L) - 1ull);
  for (int r = 0; r < 64 && msect_fits(t.lo, t.hi, L); ++r) {
    const bool above = lmax_above<N>(t, msect_point(t.lo, t.hi, lane, L));
    const unsigned long long m = (__ballot(above) >> base) & gm;
    msect_update(t.lo, t.hi, m, L);
  }
  return lmax_finish<N>(t);
}

template <int L>
__device__ inline double lambda_max_sym_lanes(const double* G, int n, int lane, int base) {
  double r = 0.0;
  LRADI_SMALL_SWITCH(n, r = (lambda_max_sym_lanes_t<NN, L>(G, lane, base)));
  return r;
}

}  // namespace lradi
