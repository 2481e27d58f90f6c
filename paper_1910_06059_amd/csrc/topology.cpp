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

extern "C" int opm_topology_build(int32_t nx, int32_t ny, int32_t nz, const uint8_t* mask,
                                  opm_topology* t) {
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
  std::vector<int32_t> level(n, 0), hmap(nx + ny + nz, -1);
  for (int32_t ci = 0; ci < n; ++ci) {
    const int32_t b = t->cell_box[ci];
    hmap[b % nx + (b / nx) % ny + b / (nx * ny)] = 0;
  }
  int32_t nlev = 0;
  for (auto& h : hmap)
    if (h == 0) h = nlev++;
  for (int32_t ci = 0; ci < n; ++ci) {
    const int32_t b = t->cell_box[ci];
    level[ci] = hmap[b % nx + (b / nx) % ny + b / (nx * ny)];
  }
  std::vector<int32_t> cnt(nlev + 1, 0);
  for (int32_t ci = 0; ci < n; ++ci) cnt[level[ci] + 1]++;
  int32_t mx = 0;
  for (int32_t l = 0; l < nlev; ++l) {
    mx = std::max(mx, cnt[l + 1]);
    cnt[l + 1] += cnt[l];
  }
  for (int32_t l = 0; l <= nlev; ++l) t->level_ptr[l] = cnt[l];
  for (int32_t ci = 0; ci < n; ++ci) {   // ascending cell order within a level
    int32_t pos = cnt[level[ci]]++;
    t->perm[pos] = ci;
    t->iperm[ci] = pos;
  }
  for (int32_t pos = 0; pos < n; ++pos) {
    int32_t ci = t->perm[pos];
    int32_t s = 0;
    for (int32_t r = t->row_ptr[ci]; r < t->diag_pos[ci]; ++r, ++s) {
      int32_t kc = t->col_idx[r];
      t->lo_blk[3 * pos + s] = r;
      t->lo_pos[3 * pos + s] = t->iperm[kc];
      int32_t tb = -1;   // block (k, i) in row k
      for (int32_t r2 = t->diag_pos[kc] + 1; r2 < t->row_ptr[kc + 1]; ++r2)
        if (t->col_idx[r2] == ci) tb = r2;
      t->lo_tblk[3 * pos + s] = tb;
    }
    for (; s < 3; ++s) t->lo_blk[3 * pos + s] = t->lo_tblk[3 * pos + s] = t->lo_pos[3 * pos + s] = -1;
    s = 0;
    for (int32_t r = t->diag_pos[ci] + 1; r < t->row_ptr[ci + 1]; ++r, ++s) {
      t->up_blk[3 * pos + s] = r;
      t->up_pos[3 * pos + s] = t->iperm[t->col_idx[r]];
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
