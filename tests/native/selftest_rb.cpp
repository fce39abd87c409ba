// Host build of the red-black preconditioner tables (colouring, slot
// tables, Schur pattern, tiles and halos) for the CPU tests; the tables are
// built once per call of st_rb_build and copied out by name.
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "../../paper_2312_02891_amd/csrc/rbhost.h"

namespace lradi {
void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vfprintf(stderr, fmt, ap);
  va_end(ap);
}
void csr_transpose(int n, const int32_t* rp, const int32_t* ci, const double* v, std::vector<int32_t>& trp,
                   std::vector<int32_t>& tci, std::vector<double>& tv);
}  // namespace lradi

static lradi::RbHost g_h;

extern "C" {
// 1 on success, 0 when the graph is not bipartite; info: nred, rbw, t2w,
// tile, ntile, maxreg, halo entries
int st_rb_build(int n, const int32_t* rp, const int32_t* ci, const double* v, int tiles, int32_t* info) {
  std::vector<int32_t> trp, tci;
  std::vector<double> tv;
  lradi::csr_transpose(n, rp, ci, v, trp, tci, tv);
  g_h = lradi::RbHost{};
  if (!lradi::rb_host_build(n, rp, ci, v, trp.data(), tci.data(), tv.data(), tiles, g_h)) return 0;
  const int32_t x[7] = {g_h.nred, g_h.rbw, g_h.t2w, g_h.tile, g_h.ntile, g_h.maxreg, (int32_t)g_h.halo.size()};
  std::memcpy(info, x, sizeof(x));
  return 1;
}
// integer tables: rows, pos, eci, t2ci, t2rev, t2lc, halo_off, halo, halo_ci; returns the
// length (dst may be null to ask for it)
long st_rb_ints(const char* name, int32_t* dst) {
  const std::vector<int32_t>* v = nullptr;
  if (!std::strcmp(name, "rows")) v = &g_h.rows;
  else if (!std::strcmp(name, "pos")) v = &g_h.pos;
  else if (!std::strcmp(name, "eci")) v = &g_h.eci;
  else if (!std::strcmp(name, "t2ci")) v = &g_h.t2ci;
  else if (!std::strcmp(name, "t2rev")) v = &g_h.t2rev;
  else if (!std::strcmp(name, "t2lc")) v = &g_h.t2lc;
  else if (!std::strcmp(name, "halo_off")) v = &g_h.halo_off;
  else if (!std::strcmp(name, "halo")) v = &g_h.halo;
  else if (!std::strcmp(name, "halo_ci")) v = &g_h.halo_ci;
  if (!v) return -1;
  if (dst) std::memcpy(dst, v->data(), sizeof(int32_t) * v->size());
  return (long)v->size();
}
// FP64 tables: dg, eval, etv
long st_rb_doubles(const char* name, double* dst) {
  const std::vector<double>* v = nullptr;
  if (!std::strcmp(name, "dg")) v = &g_h.dg;
  else if (!std::strcmp(name, "eval")) v = &g_h.eval;
  else if (!std::strcmp(name, "etv")) v = &g_h.etv;
  if (!v) return -1;
  if (dst) std::memcpy(dst, v->data(), sizeof(double) * v->size());
  return (long)v->size();
}
}
