// Host planner: truncated cluster, first neighbours and short/long regions of every atom
// (Sec. III, steps (i)-(iv)), plus the index tables the kernels read.  The sphere search runs
// over a cell list (O(N) for a fixed radius).
//
// Rules (the same readings the CPU oracle states):
//  * distances are minimum-image distances along periodic axes of an orthorhombic cell;
//    every atom appears at most once in a cluster;
//  * cluster C_i = {j : dist(i,j) <= r_L (1 + tol)} (inclusive sphere);
//  * F_i = pattern row of i (the structural overlap neighbours), always kept in the short
//    region;
//  * shells = maximal runs of equal distance; the short region is the smallest shell
//    prefix holding >= N_F + kappa (N_C - N_F) atoms; the long region is the rest.
// Library member order: long atoms, short atoms outside F_i, F_i without i, then i (each
// group by distance, then index).  With F_i last the density rows only need the trailing
// rows of the cluster problem; with i last its inverse-Cholesky columns are one block.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "ldc_internal.h"

namespace ldc {

ldc_status build_regions(Plan &p, const double *pos, const double *cell, const int *periodic) {
  const int n = p.n_atoms;
  const double r_L = p.opt.r_L;
  const double dtol = (p.opt.dist_tol > 0 ? p.opt.dist_tol : 1e-9) * std::max(1.0, r_L);
  const double stol = (p.opt.shell_tol > 0 ? p.opt.shell_tol : 1e-8) * std::max(1.0, r_L);
  const double kappa = p.opt.kappa >= 0 ? p.opt.kappa : 0.3;
  double len[3] = {cell[0], cell[4], cell[8]};

  p.mem_ptr.assign(n + 1, 0);
  p.mem_atom.clear();
  p.mem_long.clear();
  p.pair_ptr.assign(n + 1, 0);
  p.pair_ab.clear();
  p.pair_blk.clear();
  p.fna_ptr.assign(n + 1, 0);
  p.fna_blk.clear();
  p.p_rows.assign(n, 0);
  p.dmax.assign(n, 0);
  p.max_members = 0;
  p.max_dim = 0;

  // Cell list: along every axis cells of width >= the search radius (periodic axes: the cell
  // length divided evenly; open axes: from the smallest coordinate), so every atom within the
  // radius of i lies in i's cell or a neighbouring one.  Neighbour cells along an axis are
  // deduplicated (a periodic axis with fewer than three cells is searched whole), and the
  // distance test is the minimum-image test of every candidate, so the cluster is exactly
  // {j : dist(i, j) <= r_L (1 + tol)} whatever the cell sizes.
  const double rc = r_L + dtol;
  int ncell[3];
  double lo[3], width[3];
  for (int ax = 0; ax < 3; ++ax) {
    if (periodic[ax]) {
      lo[ax] = 0.0;
      ncell[ax] = std::max(1, (int)std::floor(len[ax] / rc));
      width[ax] = len[ax] / ncell[ax];
    } else {
      double mn = pos[ax], mx = pos[ax];
      for (int j = 1; j < n; ++j) {
        mn = std::min(mn, pos[3 * j + ax]);
        mx = std::max(mx, pos[3 * j + ax]);
      }
      lo[ax] = mn;
      width[ax] = rc;
      ncell[ax] = std::max(1, (int)std::floor((mx - mn) / rc) + 1);
    }
    ncell[ax] = std::min(ncell[ax], 1 << 10);
  }
  auto cell_of = [&](int j, int ax) {
    double x = pos[3 * j + ax] - lo[ax];
    if (periodic[ax]) x -= len[ax] * std::floor(x / len[ax]);
    int c = (int)std::floor(x / width[ax]);
    return std::max(0, std::min(ncell[ax] - 1, c));
  };
  const long long ntot = (long long)ncell[0] * ncell[1] * ncell[2];
  std::vector<int> cell_start(ntot + 1, 0), cell_atoms(n);
  std::vector<long long> atom_cell(n);
  for (int j = 0; j < n; ++j) {
    atom_cell[j] = ((long long)cell_of(j, 0) * ncell[1] + cell_of(j, 1)) * ncell[2] + cell_of(j, 2);
    cell_start[atom_cell[j] + 1] += 1;
  }
  for (long long c = 0; c < ntot; ++c) cell_start[c + 1] += cell_start[c];
  {
    std::vector<int> fill(cell_start.begin(), cell_start.end() - 1);
    for (int j = 0; j < n; ++j) cell_atoms[fill[atom_cell[j]]++] = j;
  }
  auto neighbours = [&](int c, int ax, int *out) {
    int k = 0;
    for (int o = -1; o <= 1; ++o) {
      int cc = c + o;
      if (periodic[ax]) cc = ((cc % ncell[ax]) + ncell[ax]) % ncell[ax];
      else if (cc < 0 || cc >= ncell[ax]) continue;
      bool dup = false;
      for (int q = 0; q < k; ++q) dup |= (out[q] == cc);
      if (!dup) out[k++] = cc;
    }
    return k;
  };

  std::vector<std::pair<double, int>> cand;
  std::vector<int> stamp(n, -1), midx(n, -1);
  std::vector<char> is_fna(n, 0);
  for (int i = 0; i < n; ++i) {
    cand.clear();
    int nb[3][3], nn[3];
    for (int ax = 0; ax < 3; ++ax) nn[ax] = neighbours(cell_of(i, ax), ax, nb[ax]);
    for (int a = 0; a < nn[0]; ++a)
      for (int b = 0; b < nn[1]; ++b)
        for (int c3 = 0; c3 < nn[2]; ++c3) {
          const long long cell = ((long long)nb[0][a] * ncell[1] + nb[1][b]) * ncell[2] + nb[2][c3];
          for (int q = cell_start[cell]; q < cell_start[cell + 1]; ++q) {
            const int j = cell_atoms[q];
            double d2 = 0.0;
            for (int ax = 0; ax < 3; ++ax) {
              double dx = pos[3 * j + ax] - pos[3 * i + ax];
              if (periodic[ax]) dx -= len[ax] * std::nearbyint(dx / len[ax]);
              d2 += dx * dx;
            }
            double d = std::sqrt(d2);
            if (d <= r_L + dtol) cand.emplace_back(d, j);
          }
        }
    std::sort(cand.begin(), cand.end());
    const int nc = (int)cand.size();
    if (nc > kMaxMembers) {
      p.msg = "cluster of atom " + std::to_string(i) + " has " + std::to_string(nc) + " atoms (limit " +
              std::to_string(kMaxMembers) + ")";
      p.err_where = i;
      return LDC_ERR_LIMIT;
    }
    // first neighbours: the pattern row (and i itself)
    for (int b = p.row_ptr[i]; b < p.row_ptr[i + 1]; ++b) is_fna[p.col[b]] = 1;
    is_fna[i] = 1;
    int nf = 0;
    for (auto &c : cand) nf += is_fna[c.second];
    int nf_row = 0;
    for (int b = p.row_ptr[i]; b < p.row_ptr[i + 1]; ++b) nf_row += (p.col[b] != i);
    if (nf != nf_row + 1) {
      for (int b = p.row_ptr[i]; b < p.row_ptr[i + 1]; ++b) is_fna[p.col[b]] = 0;
      is_fna[i] = 0;
      p.msg = "pattern neighbours of atom " + std::to_string(i) + " lie outside r_L";
      p.err_where = i;
      return LDC_ERR_ARG;
    }
    // short region: smallest shell prefix with count >= N_F + kappa N_S
    const double target = nf + kappa * (nc - nf);
    int n_sphere = nc;
    for (int k = 0; k < nc; ++k) {
      bool end = (k == nc - 1) || (cand[k + 1].first > cand[k].first + stol);
      if (end && (k + 1) >= target - 1e-12) {
        n_sphere = k + 1;
        break;
      }
    }
    std::vector<int> g_long, g_short, g_fna;
    for (int k = 0; k < nc; ++k) {
      int j = cand[k].second;
      if (j == i) continue;
      if (is_fna[j])
        g_fna.push_back(j);
      else if (k < n_sphere)
        g_short.push_back(j);
      else
        g_long.push_back(j);
    }
    for (int b = p.row_ptr[i]; b < p.row_ptr[i + 1]; ++b) is_fna[p.col[b]] = 0;
    is_fna[i] = 0;

    const int base = (int)p.mem_atom.size();
    auto push = [&](int j, int lng) {
      stamp[j] = i;
      midx[j] = (int)p.mem_atom.size() - base;
      p.mem_atom.push_back(j);
      p.mem_long.push_back(lng);
    };
    for (int j : g_long) push(j, 1);
    for (int j : g_short) push(j, 0);
    for (int j : g_fna) push(j, 0);
    push(i, 0);
    p.mem_ptr[i + 1] = (int)p.mem_atom.size();
    p.max_members = std::max(p.max_members, nc);

    // gather list: every pattern block between two members
    for (int a = 0; a < nc; ++a) {
      int ja = p.mem_atom[base + a];
      for (int b = p.row_ptr[ja]; b < p.row_ptr[ja + 1]; ++b) {
        int jb = p.col[b];
        if (stamp[jb] == i) {
          p.pair_ab.push_back(a | (midx[jb] << 16));
          p.pair_blk.push_back(b);
        }
      }
    }
    p.pair_ptr[i + 1] = (int)p.pair_ab.size();

    // P rows: F \ {i} then i; block (i, j) of row i for each
    int prow = 0;
    auto find_blk = [&](int j) {
      const int *lo = p.col.data() + p.row_ptr[i];
      const int *hi = p.col.data() + p.row_ptr[i + 1];
      const int *it = std::lower_bound(lo, hi, j);
      return (int)(it - p.col.data());
    };
    for (int j : g_fna) {
      p.fna_blk.push_back(find_blk(j));
      prow += p.n_orb[j];
    }
    p.fna_blk.push_back(find_blk(i));
    prow += p.n_orb[i];
    p.fna_ptr[i + 1] = (int)p.fna_blk.size();
    p.p_rows[i] = prow;

    int dm = 0;
    for (int a = 0; a < nc; ++a) dm += p.n_orb[p.mem_atom[base + a]];
    p.dmax[i] = dm;
    p.max_dim = std::max(p.max_dim, dm);
  }
  p.order.resize(n);
  std::iota(p.order.begin(), p.order.end(), 0);
  std::stable_sort(p.order.begin(), p.order.end(), [&](int a, int b) { return p.dmax[a] > p.dmax[b]; });
  return LDC_OK;
}

}  // namespace ldc
