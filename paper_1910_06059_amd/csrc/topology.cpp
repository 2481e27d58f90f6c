// Host-side set-up of a masked Cartesian box: active-cell numbering, the
// connection set C(i) (paper sec. 2.1.1), the 3x3-block CSR pattern of the
// Jacobian (sec. 2.3.1, block matrix storage) and the ILU(0) level schedule.
// Integer graph work done once per case; no floating point here.
#include <algorithm>
#include <cstring>
#include <vector>

#include "opm_gpu.h"

namespace {

struct Box {
  int nx, ny, nz;
  long nb() const { return (long)nx * ny * nz; }
};

bool active(const uint8_t* mask, long b) { return mask == nullptr || mask[b] != 0; }

}  // namespace

extern "C" int opm_topology_count(int32_t nx, int32_t ny, int32_t nz, const uint8_t* mask,
                                  int32_t* n_cells, int32_t* n_faces) {
  if (nx <= 0 || ny <= 0 || nz <= 0 || !n_cells || !n_faces) return OPM_EINVAL;
  Box bx{nx, ny, nz};
  if (bx.nb() >= (1L << 30)) return OPM_EINVAL;
  long n = 0, nf = 0;
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        long b = i + (long)nx * (j + (long)ny * k);
        if (!active(mask, b)) continue;
        ++n;
        if (i + 1 < nx && active(mask, b + 1)) ++nf;
        if (j + 1 < ny && active(mask, b + nx)) ++nf;
        if (k + 1 < nz && active(mask, b + (long)nx * ny)) ++nf;
      }
  *n_cells = (int32_t)n;
  *n_faces = (int32_t)nf;
  return OPM_OK;
}

namespace {

// Subdomain boxes of the block ILU0 (paper sec. 2.5: one block per process):
// box (i / bx, j / by, k / bz); boxes without active cells are dropped and
// the others numbered densely in box order.  Level of a cell: the local
// hyperplane (i mod bx) + (j mod by) + (k mod bz), densely numbered over the
// values that hold cells, so every lower neighbour inside the subdomain lies
// on the previous level.
struct Blocking {
  int bx, by, bz;
  std::vector<int32_t> sub;   // [n] dense subdomain of each cell
  int32_t n_sub = 0;
};

int blocking_of(int nx, int ny, int nz, const uint8_t* mask, int bx, int by, int bz,
                Blocking& B) {
  if (bx <= 0 || by <= 0 || bz <= 0) return OPM_EINVAL;
  // a box longer than the grid is the whole axis
  bx = std::min(bx, nx);
  by = std::min(by, ny);
  bz = std::min(bz, nz);
  B.bx = bx;
  B.by = by;
  B.bz = bz;
  const long nbx = (nx + bx - 1) / bx, nby = (ny + by - 1) / by, nbz = (nz + bz - 1) / bz;
  std::vector<int32_t> box_sub(nbx * nby * nbz, -1);
  B.sub.clear();
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        const long b = i + (long)nx * (j + (long)ny * k);
        if (!active(mask, b)) continue;
        const long q = i / bx + nbx * (j / by + nby * (k / bz));
        box_sub[q] = 0;
      }
  B.n_sub = 0;
  for (auto& q : box_sub)
    if (q == 0) q = B.n_sub++;
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        const long b = i + (long)nx * (j + (long)ny * k);
        if (active(mask, b)) B.sub.push_back(box_sub[i / bx + nbx * (j / by + nby * (k / bz))]);
      }
  return OPM_OK;
}

int build(int32_t nx, int32_t ny, int32_t nz, const uint8_t* mask, const Blocking* B,
          opm_ilu_blocks* blk, opm_topology* t);

}  // namespace

extern "C" int opm_topology_build(int32_t nx, int32_t ny, int32_t nz, const uint8_t* mask,
                                  opm_topology* t) {
  return build(nx, ny, nz, mask, nullptr, nullptr, t);
}

extern "C" int opm_ilu_blocks_count(int32_t nx, int32_t ny, int32_t nz, const uint8_t* mask,
                                    int32_t bx, int32_t by, int32_t bz, int32_t* n_sub,
                                    int32_t* n_levels) {
  int32_t n = 0, nf = 0;
  int st = opm_topology_count(nx, ny, nz, mask, &n, &nf);
  if (st != OPM_OK) return st;
  if (!n_sub || !n_levels) return OPM_EINVAL;
  Blocking B;
  st = blocking_of(nx, ny, nz, mask, bx, by, bz, B);
  if (st != OPM_OK) return st;
  std::vector<char> h((size_t)B.bx + B.by + B.bz, 0);
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i)
        if (active(mask, i + (long)nx * (j + (long)ny * k))) h[i % B.bx + j % B.by + k % B.bz] = 1;
  int32_t nl = 0;
  for (char c : h) nl += c;
  *n_sub = B.n_sub;
  *n_levels = nl;
  return OPM_OK;
}

extern "C" int opm_topology_build_blocks(int32_t nx, int32_t ny, int32_t nz, const uint8_t* mask,
                                         opm_ilu_blocks* blk, opm_topology* t) {
  if (!blk || !blk->sub_level_ptr || !blk->slot) return OPM_EINVAL;
  int32_t n = 0, nf = 0;
  int st = opm_topology_count(nx, ny, nz, mask, &n, &nf);
  if (st != OPM_OK) return st;
  Blocking B;
  st = blocking_of(nx, ny, nz, mask, blk->bx, blk->by, blk->bz, B);
  if (st != OPM_OK) return st;
  return build(nx, ny, nz, mask, &B, blk, t);
}

namespace {

int build(int32_t nx, int32_t ny, int32_t nz, const uint8_t* mask, const Blocking* B,
          opm_ilu_blocks* blk, opm_topology* t) {
  int32_t n = 0, nf = 0;
  int st = opm_topology_count(nx, ny, nz, mask, &n, &nf);
  if (st != OPM_OK) return st;
  if (!t || !t->cell_box || !t->face_cells || !t->face_dir || !t->row_ptr || !t->col_idx ||
      !t->blk_face || !t->diag_pos || !t->level_ptr || !t->perm || !t->iperm || !t->lo_blk ||
      !t->lo_tblk || !t->lo_pos || !t->up_blk || !t->up_pos)
    return OPM_EINVAL;
  Box bx{nx, ny, nz};
  const long sxy = (long)nx * ny;
  std::vector<int32_t> box_cell(bx.nb(), -1);
  int32_t c = 0;
  for (long b = 0; b < bx.nb(); ++b)
    if (active(mask, b)) {
      box_cell[b] = c;
      t->cell_box[c] = (int32_t)b;
      ++c;
    }
  // faces owned by their lower cell: +x, +y, +z neighbours
  std::vector<int32_t> face_plus((size_t)n * 3, -1);
  int32_t f = 0;
  for (int32_t ci = 0; ci < n; ++ci) {
    long b = t->cell_box[ci];
    int i = (int)(b % nx), j = (int)((b / nx) % ny), k = (int)(b / sxy);
    const long nbr[3] = {b + 1, b + nx, b + sxy};
    const bool inside[3] = {i + 1 < nx, j + 1 < ny, k + 1 < nz};
    for (int d = 0; d < 3; ++d) {
      if (!inside[d] || box_cell[nbr[d]] < 0) continue;
      t->face_cells[2 * f] = ci;
      t->face_cells[2 * f + 1] = box_cell[nbr[d]];
      t->face_dir[f] = d;
      face_plus[(size_t)ci * 3 + d] = f;
      ++f;
    }
  }
  // block rows: columns in ascending order -z, -y, -x, self, +x, +y, +z
  int32_t q = 0;
  for (int32_t ci = 0; ci < n; ++ci) {
    long b = t->cell_box[ci];
    int i = (int)(b % nx), j = (int)((b / nx) % ny), k = (int)(b / sxy);
    t->row_ptr[ci] = q;
    const long lower[3] = {b - sxy, b - nx, b - 1};
    const bool lin[3] = {k > 0, j > 0, i > 0};
    const int ldir[3] = {2, 1, 0};
    for (int s = 0; s < 3; ++s) {
      if (!lin[s] || box_cell[lower[s]] < 0) continue;
      int32_t nbc = box_cell[lower[s]];
      t->col_idx[q] = nbc;
      t->blk_face[q] = face_plus[(size_t)nbc * 3 + ldir[s]];
      ++q;
    }
    t->diag_pos[ci] = q;
    t->col_idx[q] = ci;
    t->blk_face[q] = -1;
    ++q;
    for (int d = 0; d < 3; ++d) {
      int32_t fp = face_plus[(size_t)ci * 3 + d];
      if (fp < 0) continue;
      t->col_idx[q] = t->face_cells[2 * fp + 1];
      t->blk_face[q] = fp;
      ++q;
    }
  }
  t->row_ptr[n] = q;

  // ILU(0) level schedule: the hyperplanes i + j + k = h that hold active
  // cells, in increasing h.  Every lower neighbour of a cell lies on h - 1,
  // i.e. on the previous level, so rows of one level are independent and a
  // sweep needs the values of two consecutive levels only (on a masked grid
  // the as-soon-as-possible schedule would put neighbours many levels apart).
  // With subdomains: the local hyperplanes, and inside a level the rows
  // grouped by subdomain (positions ordered by level, subdomain, cell).
  const int hx = B ? B->bx : nx, hy = B ? B->by : ny, hz = B ? B->bz : nz;
  const int32_t nsub = B ? B->n_sub : 1;
  auto hyper = [&](int32_t b) { return b % nx % hx + (b / nx) % ny % hy + b / (nx * ny) % hz; };
  auto sub_of = [&](int32_t ci) { return B ? B->sub[ci] : 0; };
  std::vector<int32_t> level(n, 0), hmap((size_t)hx + hy + hz, -1);
  for (int32_t ci = 0; ci < n; ++ci) hmap[hyper(t->cell_box[ci])] = 0;
  int32_t nlev = 0;
  for (auto& h : hmap)
    if (h == 0) h = nlev++;
  for (int32_t ci = 0; ci < n; ++ci) level[ci] = hmap[hyper(t->cell_box[ci])];
  // counting sort over the key (level, subdomain)
  std::vector<int32_t> cnt((size_t)nlev * nsub + 1, 0);
  for (int32_t ci = 0; ci < n; ++ci) cnt[(size_t)level[ci] * nsub + sub_of(ci) + 1]++;
  int32_t mw = 0;
  for (size_t q = 0; q + 1 < cnt.size(); ++q) {
    mw = std::max(mw, cnt[q + 1]);
    cnt[q + 1] += cnt[q];
  }
  int32_t mx = 0;
  for (int32_t l = 0; l <= nlev; ++l) t->level_ptr[l] = cnt[(size_t)l * nsub];
  for (int32_t l = 0; l < nlev; ++l) mx = std::max(mx, t->level_ptr[l + 1] - t->level_ptr[l]);
  if (B) {
    for (int32_t l = 0; l < nlev; ++l)
      for (int32_t sb = 0; sb <= nsub; ++sb)
        blk->sub_level_ptr[(size_t)l * (nsub + 1) + sb] = cnt[(size_t)l * nsub + sb];
  }
  std::vector<int32_t> start(cnt.begin(), cnt.end() - 1);
  for (int32_t ci = 0; ci < n; ++ci) {   // ascending cell order within a key
    int32_t pos = start[(size_t)level[ci] * nsub + sub_of(ci)]++;
    t->perm[pos] = ci;
    t->iperm[ci] = pos;
  }
  if (B) {
    // slot: index of a row inside its subdomain (levels ascending)
    std::vector<int32_t> fill(nsub, 0);
    int32_t ms = 0;
    for (int32_t l = 0; l < nlev; ++l)
      for (int32_t sb = 0; sb < nsub; ++sb) {
        const int32_t p0 = cnt[(size_t)l * nsub + sb], p1 = cnt[(size_t)l * nsub + sb + 1];
        for (int32_t pos = p0; pos < p1; ++pos) blk->slot[pos] = fill[sb] + (pos - p0);
        fill[sb] += p1 - p0;
        ms = std::max(ms, fill[sb]);
      }
    blk->n_sub = nsub;
    blk->max_sub = ms;
    blk->max_width = mw;
  }
  // neighbour lists of the ILU structure: with subdomains, only neighbours
  // in the same subdomain (the couplings between subdomains are dropped)
  for (int32_t pos = 0; pos < n; ++pos) {
    int32_t ci = t->perm[pos];
    int32_t s = 0;
    for (int32_t r = t->row_ptr[ci]; r < t->diag_pos[ci]; ++r) {
      int32_t kc = t->col_idx[r];
      if (sub_of(kc) != sub_of(ci)) continue;
      t->lo_blk[3 * pos + s] = r;
      t->lo_pos[3 * pos + s] = t->iperm[kc];
      int32_t tb = -1;   // block (k, i) in row k
      for (int32_t r2 = t->diag_pos[kc] + 1; r2 < t->row_ptr[kc + 1]; ++r2)
        if (t->col_idx[r2] == ci) tb = r2;
      t->lo_tblk[3 * pos + s] = tb;
      ++s;
    }
    for (; s < 3; ++s) t->lo_blk[3 * pos + s] = t->lo_tblk[3 * pos + s] = t->lo_pos[3 * pos + s] = -1;
    s = 0;
    for (int32_t r = t->diag_pos[ci] + 1; r < t->row_ptr[ci + 1]; ++r) {
      if (sub_of(t->col_idx[r]) != sub_of(ci)) continue;
      t->up_blk[3 * pos + s] = r;
      t->up_pos[3 * pos + s] = t->iperm[t->col_idx[r]];
      ++s;
    }
    for (; s < 3; ++s) t->up_blk[3 * pos + s] = t->up_pos[3 * pos + s] = -1;
  }
  int32_t span = 0;
  for (int32_t pos = 0; pos < n; ++pos)
    for (int s2 = 0; s2 < 3; ++s2) {
      if (t->lo_pos[3 * pos + s2] >= 0) span = std::max(span, pos - t->lo_pos[3 * pos + s2]);
      if (t->up_pos[3 * pos + s2] >= 0) span = std::max(span, t->up_pos[3 * pos + s2] - pos);
    }
  t->n_levels = nlev;
  t->max_level = mx;
  t->sweep_span = span;
  return OPM_OK;
}

}  // namespace

extern "C" int opm_well_groups(int32_t n_cells, int32_t n_conns, const int32_t* conn_cell,
                               int32_t* cell_conn_ptr, int32_t* cell_conn) {
  if (n_cells < 0 || n_conns < 0 || !cell_conn_ptr || (n_conns > 0 && (!conn_cell || !cell_conn)))
    return OPM_EINVAL;
  for (int32_t k = 0; k < n_conns; ++k)
    if (conn_cell[k] < 0 || conn_cell[k] >= n_cells) return OPM_EINVAL;
  std::vector<int32_t> cnt((size_t)n_cells + 1, 0);
  for (int32_t k = 0; k < n_conns; ++k) cnt[conn_cell[k] + 1]++;
  for (int32_t c = 0; c < n_cells; ++c) cnt[c + 1] += cnt[c];
  for (int32_t c = 0; c <= n_cells; ++c) cell_conn_ptr[c] = cnt[c];
  for (int32_t k = 0; k < n_conns; ++k) cell_conn[cnt[conn_cell[k]]++] = k;
  return OPM_OK;
}

// ---------------------------------------------------------------- CPR-AMG
// The aggregation hierarchy of the CPR pressure stage: geometric 2x2x2
// aggregates of each level's lattice, the coarse patterns, and the gather
// maps of the Galerkin products.  Built level by level; count and build run
// the same construction (count keeps only the sizes).
namespace {

struct AmgLevel {
  int dims[3];
  std::vector<int> box;                // lattice box of each unknown
  std::vector<int32_t> row_ptr, col, dpos;
  std::vector<int32_t> agg, child_ptr, child;   // to the next level
  std::vector<int32_t> gmap_ptr, gmap;           // from the previous level
};

int amg_hierarchy(int nx, int ny, int nz, const uint8_t* mask, int n, const int32_t* row_ptr,
                  const int32_t* col_idx, std::vector<AmgLevel>& L) {
  L.clear();
  L.emplace_back();
  AmgLevel& l0 = L.back();
  l0.dims[0] = nx;
  l0.dims[1] = ny;
  l0.dims[2] = nz;
  l0.box.reserve(n);
  for (long b = 0; b < (long)nx * ny * nz; ++b)
    if (active(mask, b)) l0.box.push_back((int)b);
  if ((int)l0.box.size() != n) return OPM_EINVAL;
  l0.row_ptr.assign(row_ptr, row_ptr + n + 1);
  l0.col.assign(col_idx, col_idx + row_ptr[n]);
  while ((int)L.back().box.size() > OPM_AMG_COARSE && (int)L.size() < OPM_AMG_MAX_LEVELS) {
    AmgLevel& f = L.back();
    const int* d = f.dims;
    if (d[0] == 1 && d[1] == 1 && d[2] == 1) break;
    const int cd[3] = {(d[0] + 1) / 2, (d[1] + 1) / 2, (d[2] + 1) / 2};
    const long nbc = (long)cd[0] * cd[1] * cd[2];
    const int nf = (int)f.box.size();
    std::vector<int> idx(nbc, -1), parent(nf);
    for (int i = 0; i < nf; ++i) {
      const int b = f.box[i];
      const int x = b % d[0], y = (b / d[0]) % d[1], z = b / (d[0] * d[1]);
      parent[i] = x / 2 + cd[0] * (y / 2 + cd[1] * (z / 2));
      idx[parent[i]] = 0;
    }
    AmgLevel c;
    int nc = 0;
    for (long b = 0; b < nbc; ++b)
      if (idx[b] >= 0) {
        idx[b] = nc++;
        c.box.push_back((int)b);
      }
    std::memcpy(c.dims, cd, sizeof cd);
    f.agg.resize(nf);
    for (int i = 0; i < nf; ++i) f.agg[i] = idx[parent[i]];
    f.child_ptr.assign(nc + 1, 0);
    for (int i = 0; i < nf; ++i) f.child_ptr[f.agg[i] + 1]++;
    for (int I = 0; I < nc; ++I) f.child_ptr[I + 1] += f.child_ptr[I];
    f.child.resize(nf);
    {
      std::vector<int32_t> fill(f.child_ptr.begin(), f.child_ptr.end() - 1);
      for (int i = 0; i < nf; ++i) f.child[fill[f.agg[i]]++] = i;
    }
    // coarse rows: the aggregates of the children's columns, ascending; each
    // coarse entry gathers its fine entries in the order children, entries
    c.row_ptr.assign(nc + 1, 0);
    std::vector<std::vector<int32_t>> members;
    for (int I = 0; I < nc; ++I) {
      std::vector<std::pair<int32_t, int32_t>> e;   // (coarse column, fine entry)
      for (int t = f.child_ptr[I]; t < f.child_ptr[I + 1]; ++t) {
        const int i = f.child[t];
        for (int q = f.row_ptr[i]; q < f.row_ptr[i + 1]; ++q) e.push_back({f.agg[f.col[q]], q});
      }
      std::stable_sort(e.begin(), e.end(),
                       [](const std::pair<int32_t, int32_t>& a,
                          const std::pair<int32_t, int32_t>& b) { return a.first < b.first; });
      for (size_t u = 0; u < e.size(); ++u) {
        if (u == 0 || e[u].first != e[u - 1].first) {
          c.col.push_back(e[u].first);
          members.emplace_back();
        }
        members.back().push_back(e[u].second);
      }
      c.row_ptr[I + 1] = (int32_t)c.col.size();
    }
    c.gmap_ptr.assign(members.size() + 1, 0);
    for (size_t k = 0; k < members.size(); ++k) {
      c.gmap_ptr[k + 1] = c.gmap_ptr[k] + (int32_t)members[k].size();
      c.gmap.insert(c.gmap.end(), members[k].begin(), members[k].end());
    }
    c.dpos.resize(nc);
    for (int I = 0; I < nc; ++I)
      for (int q = c.row_ptr[I]; q < c.row_ptr[I + 1]; ++q)
        if (c.col[q] == I) c.dpos[I] = q;
    L.push_back(std::move(c));
  }
  // the coarsest level is solved by its dense inverse
  if ((int)L.back().box.size() > OPM_AMG_COARSE) return OPM_EINVAL;
  return OPM_OK;
}

int amg_fill(int nx, int ny, int nz, const uint8_t* mask, int n, const int32_t* row_ptr,
             const int32_t* col_idx, opm_amg* out, bool arrays) {
  if (nx <= 0 || ny <= 0 || nz <= 0 || n <= 0 || !row_ptr || !col_idx || !out) return OPM_EINVAL;
  std::vector<AmgLevel> L;
  const int st = amg_hierarchy(nx, ny, nz, mask, n, row_ptr, col_idx, L);
  if (st != OPM_OK) return st;
  out->n_levels = (int32_t)L.size();
  for (size_t l = 0; l < L.size(); ++l) {
    out->n[l] = (int32_t)L[l].box.size();
    out->nnz[l] = (int32_t)L[l].col.size();
  }
  if (!arrays) return OPM_OK;
  auto put = [](int32_t* dst, const std::vector<int32_t>& v) {
    if (!v.empty()) std::memcpy(dst, v.data(), sizeof(int32_t) * v.size());
  };
  for (size_t l = 0; l < L.size(); ++l) {
    if (l >= 1) {
      if (!out->row_ptr[l] || !out->col[l] || !out->dpos[l] || !out->gmap_ptr[l] || !out->gmap[l])
        return OPM_EINVAL;
      put(out->row_ptr[l], L[l].row_ptr);
      put(out->col[l], L[l].col);
      put(out->dpos[l], L[l].dpos);
      put(out->gmap_ptr[l], L[l].gmap_ptr);
      put(out->gmap[l], L[l].gmap);
    }
    if (l + 1 < L.size()) {
      if (!out->agg[l] || !out->child_ptr[l] || !out->child[l]) return OPM_EINVAL;
      put(out->agg[l], L[l].agg);
      put(out->child_ptr[l], L[l].child_ptr);
      put(out->child[l], L[l].child);
    }
  }
  return OPM_OK;
}

}  // namespace

extern "C" int opm_amg_count(int32_t nx, int32_t ny, int32_t nz, const uint8_t* mask,
                             int32_t n_cells, const int32_t* row_ptr, const int32_t* col_idx,
                             opm_amg* out) {
  return amg_fill(nx, ny, nz, mask, n_cells, row_ptr, col_idx, out, false);
}

extern "C" int opm_amg_build(int32_t nx, int32_t ny, int32_t nz, const uint8_t* mask,
                             int32_t n_cells, const int32_t* row_ptr, const int32_t* col_idx,
                             opm_amg* out) {
  return amg_fill(nx, ny, nz, mask, n_cells, row_ptr, col_idx, out, true);
}
