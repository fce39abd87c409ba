// Host construction of the red-black ILU(0) preconditioner tables (plain
// C++, no HIP, so the CPU tests build and check it too): the 2-colouring of
// the sparsity graph, A's off-diagonal entries by colour position, the
// column pattern of the Schur complement T = D_b - F D_r^{-1} E on the black
// rows, and a tiling of the black positions with halos that lets one launch
// run two Jacobi sweeps on T, the first into workgroup-local memory.
#pragma once

#include <algorithm>
#include <cstdint>
#include <thread>
#include <vector>

namespace lradi {

// f(begin, end, thread) over [0, n) split across a few host threads (one
// range when n is small)
template <class F>
void par_ranges(int n, F f) {
  const int nt = std::max(1, std::min(8, (int)std::thread::hardware_concurrency()));
  if (n < 32768 || nt == 1) {
    f(0, n, 0);
    return;
  }
  std::vector<std::thread> th;
  const int chunk = (n + nt - 1) / nt;
  for (int t = 0; t < nt; ++t) th.emplace_back(f, std::min(n, t * chunk), std::min(n, (t + 1) * chunk), t);
  for (auto& x : th) x.join();
}
inline int par_threads(int n) {
  const int nt = std::max(1, std::min(8, (int)std::thread::hardware_concurrency()));
  return n < 32768 ? 1 : nt;
}

struct RbHost {
  int nred = 0;  // red rows
  int rbw = 0;   // off-diagonal slots per row (at least 1)
  int t2w = 0;   // off-diagonal slots of T per black row (at least 1)
  // colour order: red rows ascending, then the black rows tile by tile
  // (ascending within a tile; ascending overall without tiles);
  // pos[row] = its colour position
  std::vector<int32_t> rows, pos;
  std::vector<double> dg;  // A's diagonal per row
  // slot u of colour position p at u * n + p: column, a_(i,col), a_(col,i);
  // unused slots hold the row itself with values 0
  std::vector<int32_t> eci;
  std::vector<double> eval, etv;
  // T's off-diagonal columns as black positions (pb = p - nred), slot q of
  // pb at q * max(nb, 1) + pb, in order of first appearance along the two
  // hops i -> red j -> black l; unused slots hold pb itself
  std::vector<int32_t> t2ci;
  // t2rev: for slot q of pb with column c != pb, the slot of c whose column
  // is pb (T_c,pb beside T_pb,c), slot-major like t2ci; -1 for unused slots
  // and where c has no such slot
  std::vector<int32_t> t2rev;
  // tiles: tile t holds the black positions [t * tile, min(nb, (t + 1) *
  // tile)), grown breadth first over T's graph so that it is compact; its
  // halo is the black positions outside it that its rows' T columns reach,
  // ascending, at halo[halo_off[t] .. halo_off[t + 1]).  t2lc: T's columns
  // (slot-major like t2ci) as indices into the region of the row's tile,
  // its rows first (index pb - t * tile), then its halo in order
  int tile = 0, ntile = 0;
  int maxreg = 0;  // largest region (rows + halo) of a tile
  std::vector<int32_t> halo_off, halo, t2lc;
  // the halo rows' T columns (as black positions), slot q of halo entry g
  // at q * max(nhalo, 1) + g: a halo row's gathers need not wait for its
  // position
  std::vector<int32_t> halo_ci;
};

// Fills h for the n x n CSR matrix (rp, ci, v) with transpose (trp, tci, tv)
// and `tiles` tiles of ceil(nb / tiles) black positions; tiles = 0: the
// black rows stay in ascending order and no tiles are made.
// Returns false when the sparsity graph (A and A^T, stored zeros included)
// is not bipartite.
inline bool rb_host_build(int n, const int32_t* rp, const int32_t* ci, const double* v, const int32_t* trp,
                          const int32_t* tci, const double* tv, int tiles, RbHost& h) {
  // breadth-first 2-colouring over the union of A's and A^T's off-diagonal
  // patterns, the lowest row of each component red
  std::vector<int8_t> col(n, -1);
  std::vector<int32_t> queue(n);
  for (int s0 = 0; s0 < n; ++s0) {
    if (col[s0] >= 0) continue;
    col[s0] = 0;
    int head = 0, tail = 0;
    queue[tail++] = s0;
    while (head < tail) {
      const int u = queue[head++];
      for (int pass = 0; pass < 2; ++pass) {
        const int32_t* R = pass ? trp : rp;
        const int32_t* C = pass ? tci : ci;
        for (int32_t k = R[u]; k < R[u + 1]; ++k) {
          const int w = C[k];
          if (w == u) continue;
          if (col[w] < 0) {
            col[w] = (int8_t)(1 - col[u]);
            queue[tail++] = w;
          } else if (col[w] == col[u]) {
            return false;
          }
        }
      }
    }
  }
  std::vector<int32_t> rows;
  rows.reserve(n);
  for (int i = 0; i < n; ++i)
    if (col[i] == 0) rows.push_back(i);
  const int nr = (int)rows.size();
  for (int i = 0; i < n; ++i)
    if (col[i] == 1) rows.push_back(i);
  const int nbk = n - nr;
  const size_t nbs = (size_t)std::max(nbk, 1);

  // T's columns per black row (natural black order), as rows l != i in
  // order of first appearance; slot_of[l] marks a column while its row is
  // being built.  Per-thread tables, then one flat list.
  const int nth = par_threads(nbk);
  std::vector<std::vector<int32_t>> tcols(nth);
  std::vector<std::vector<size_t>> tstart(nth);
  std::vector<int32_t> ncol(nbs, 0);
  par_ranges(nbk, [&](int pa, int pe, int t) {
    std::vector<int32_t> slot_of(n, -1);
    std::vector<int32_t>& cols = tcols[t];
    std::vector<size_t>& cs = tstart[t];
    cols.reserve((size_t)(pe - pa) * 8);
    cs.assign((size_t)(pe - pa) + 1, 0);
    for (int pb = pa; pb < pe; ++pb) {
      const int i = rows[nr + pb];
      cs[pb - pa] = cols.size();
      for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
        const int j = ci[k];
        if (j == i) continue;
        for (int32_t kk = rp[j]; kk < rp[j + 1]; ++kk) {
          const int l = ci[kk];
          if (l == j || l == i || slot_of[l] >= 0) continue;
          slot_of[l] = (int32_t)(cols.size() - cs[pb - pa]);
          cols.push_back(l);
        }
      }
      for (size_t q = cs[pb - pa]; q < cols.size(); ++q) slot_of[cols[q]] = -1;
      ncol[pb] = (int32_t)(cols.size() - cs[pb - pa]);
    }
    cs[pe - pa] = cols.size();
  });
  std::vector<int64_t> soff((size_t)nbk + 1, 0);
  for (int pb = 0; pb < nbk; ++pb) soff[pb + 1] = soff[pb] + ncol[pb];
  std::vector<int32_t> scol((size_t)soff[nbk]);
  par_ranges(nbk, [&](int pa, int pe, int t) {
    if (pe > pa) std::copy(tcols[t].begin(), tcols[t].end(), scol.begin() + soff[pa]);
  });
  tcols.clear();
  tstart.clear();
  int w2 = 0;
  for (int pb = 0; pb < nbk; ++pb) w2 = std::max(w2, ncol[pb]);
  const int W2 = std::max(w2, 1);

  // tiling: each tile grows breadth first over T's graph from the lowest
  // unassigned black row, continuing from the next seed when a component
  // runs out; its rows are then sorted by row index
  std::vector<int32_t> nat((size_t)n, -1);  // natural black position of a black row
  for (int pb = 0; pb < nbk; ++pb) nat[rows[nr + pb]] = pb;
  const int tile = (nbk > 0 && tiles > 0) ? (nbk + tiles - 1) / tiles : 0;
  std::vector<int32_t> perm(nbs);  // tile-order position -> natural position
  if (tile == 0) {
    for (int p = 0; p < nbk; ++p) perm[p] = p;
  } else {
    std::vector<uint8_t> taken(nbs, 0);
    int filled = 0, seed = 0;
    while (filled < nbk) {
      const int t0 = filled, t1 = std::min(nbk, t0 + tile);
      int head = filled;
      while (filled < t1) {
        if (head == filled) {  // queue empty: next seed
          while (taken[seed]) ++seed;
          taken[seed] = 1;
          perm[filled++] = seed;
        }
        while (head < filled && filled < t1) {
          const int u = perm[head++];
          for (int64_t k = soff[u]; k < soff[u + 1] && filled < t1; ++k) {
            const int w = nat[scol[k]];
            if (!taken[w]) {
              taken[w] = 1;
              perm[filled++] = w;
            }
          }
        }
      }
      std::sort(perm.begin() + t0, perm.begin() + t1);
    }
  }
  {
    std::vector<int32_t> brows(rows.begin() + nr, rows.end());
    for (int p = 0; p < nbk; ++p) rows[nr + p] = brows[perm[p]];
  }
  std::vector<int32_t> pos((size_t)n);
  for (int p = 0; p < n; ++p) pos[rows[p]] = p;

  // diagonal and slot tables by colour position (position-major first, then
  // a blocked transpose to slot-major)
  std::vector<double> dg(n, 0.0);
  int w = 0;
  for (int i = 0; i < n; ++i) {
    int c = 0;
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
      if (ci[k] == i) dg[i] += v[k];
      else ++c;
    }
    w = std::max(w, c);
  }
  const int W = std::max(w, 1);
  std::vector<int32_t> r_eci((size_t)W * n);
  std::vector<double> r_eval((size_t)W * n, 0.0), r_etv((size_t)W * n, 0.0);
  par_ranges(n, [&](int pa, int pe, int) {
    for (int p = pa; p < pe; ++p) {
      const int i = rows[p];
      const size_t e0 = (size_t)p * W;
      int u = 0;
      for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
        if (ci[k] == i) continue;
        double a = 0.0;
        for (int32_t kk = trp[i]; kk < trp[i + 1]; ++kk)
          if (tci[kk] == ci[k]) a += tv[kk];
        r_eci[e0 + u] = ci[k];
        r_eval[e0 + u] = v[k];
        r_etv[e0 + u] = a;
        ++u;
      }
      for (; u < W; ++u) r_eci[e0 + u] = i;
    }
  });
  h.eci.assign((size_t)W * n, 0);
  h.eval.assign((size_t)W * n, 0.0);
  h.etv.assign((size_t)W * n, 0.0);
  par_ranges(n, [&](int pa, int pe, int) {
    for (int p0 = pa; p0 < pe; p0 += 256)  // blocked: the source block stays in cache
      for (int u = 0; u < W; ++u)
        for (int p = p0; p < std::min(pe, p0 + 256); ++p) {
          h.eci[(size_t)u * n + p] = r_eci[(size_t)p * W + u];
          h.eval[(size_t)u * n + p] = r_eval[(size_t)p * W + u];
          h.etv[(size_t)u * n + p] = r_etv[(size_t)p * W + u];
        }
  });

  // T's columns as black positions in tile order
  h.t2ci.assign((size_t)W2 * nbs, 0);
  par_ranges(nbk, [&](int pa, int pe, int) {
    for (int pb = pa; pb < pe; ++pb) {
      const int old = perm[pb];
      const int64_t c0 = soff[old], nc = soff[old + 1] - c0;
      for (int q = 0; q < W2; ++q) h.t2ci[(size_t)q * nbs + pb] = q < nc ? pos[scol[c0 + q]] - nr : pb;
    }
  });

  h.t2rev.assign((size_t)W2 * nbs, -1);
  par_ranges(nbk, [&](int pa, int pe, int) {
    for (int pb = pa; pb < pe; ++pb)
      for (int q = 0; q < W2; ++q) {
        const int c = h.t2ci[(size_t)q * nbs + pb];
        if (c == pb) continue;
        for (int q2 = 0; q2 < W2; ++q2)
          if (h.t2ci[(size_t)q2 * nbs + c] == pb) {
            h.t2rev[(size_t)q * nbs + pb] = q2;
            break;
          }
      }
  });

  // halos and region-local columns, tile by tile
  const int ntile = tile > 0 ? (nbk + tile - 1) / tile : 0;
  std::vector<std::vector<int32_t>> thalo(par_threads(ntile * 256));
  std::vector<int32_t> hcount((size_t)ntile, 0);
  h.t2lc.assign((size_t)W2 * nbs, 0);
  // split the tiles over threads (by tile index, so the halo lists
  // concatenate in tile order)
  const int pt = (int)thalo.size();
  auto halo_pass = [&](int ta, int tb, int th) {
    std::vector<int32_t> loc(nbs, -1);
    std::vector<int32_t>& out = thalo[th];
    std::vector<int32_t> hl;
    for (int t = ta; t < tb; ++t) {
      const int p0 = t * tile, p1 = std::min(nbk, p0 + tile), nin = p1 - p0;
      hl.clear();
      for (int pb = p0; pb < p1; ++pb)
        for (int q = 0; q < W2; ++q) {
          const int c = h.t2ci[(size_t)q * nbs + pb];
          if ((c < p0 || c >= p1) && loc[c] < 0) {
            loc[c] = 0;
            hl.push_back(c);
          }
        }
      std::sort(hl.begin(), hl.end());
      for (size_t k = 0; k < hl.size(); ++k) loc[hl[k]] = nin + (int32_t)k;
      for (int pb = p0; pb < p1; ++pb)
        for (int q = 0; q < W2; ++q) {
          const int c = h.t2ci[(size_t)q * nbs + pb];
          h.t2lc[(size_t)q * nbs + pb] = (c >= p0 && c < p1) ? c - p0 : loc[c];
        }
      for (int32_t c : hl) loc[c] = -1;
      hcount[t] = (int32_t)hl.size();
      out.insert(out.end(), hl.begin(), hl.end());
    }
  };
  if (pt <= 1) {
    halo_pass(0, ntile, 0);
  } else {
    std::vector<std::thread> th;
    const int chunk = (ntile + pt - 1) / pt;
    for (int t = 0; t < pt; ++t)
      th.emplace_back(halo_pass, std::min(ntile, t * chunk), std::min(ntile, (t + 1) * chunk), t);
    for (auto& x : th) x.join();
  }
  h.halo_off.assign((size_t)ntile + 1, 0);
  int maxreg = 0;
  for (int t = 0; t < ntile; ++t) {
    h.halo_off[t + 1] = h.halo_off[t] + hcount[t];
    maxreg = std::max(maxreg, std::min(nbk, (t + 1) * tile) - t * tile + hcount[t]);
  }
  h.halo.clear();
  h.halo.reserve((size_t)h.halo_off[ntile]);
  for (auto& x : thalo) h.halo.insert(h.halo.end(), x.begin(), x.end());
  const size_t nh = h.halo.size(), nhs = std::max(nh, (size_t)1);
  h.halo_ci.assign((size_t)W2 * nhs, 0);
  for (int q = 0; q < W2; ++q)
    for (size_t g = 0; g < nh; ++g) h.halo_ci[(size_t)q * nhs + g] = h.t2ci[(size_t)q * nbs + h.halo[g]];

  h.nred = nr;
  h.rbw = W;
  h.t2w = W2;
  h.rows = std::move(rows);
  h.pos = std::move(pos);
  h.dg = std::move(dg);
  h.tile = tile;
  h.ntile = ntile;
  h.maxreg = maxreg;
  return true;
}

}  // namespace lradi
