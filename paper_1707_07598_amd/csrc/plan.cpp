// Host-side plan construction (see plan.hpp).
#include "plan.hpp"

#include <algorithm>
#include <cstdio>
#include <numeric>

namespace msfv {

namespace {

void make_axis(Axis& a, int n, int r) {
  a.n = n;
  a.r = r;
  a.nc = (n + r - 1) / r;
  a.v.resize(a.nc);
  for (int I = 0; I < a.nc; ++I) a.v[I] = I * r + std::min(r, n - I * r) / 2;
  a.code.assign(n, -1);
  for (int I = 0; I < a.nc; ++I) a.code[a.v[I]] = 2 * I + 1;
  for (int s = 0; s <= a.nc; ++s)
    for (int i = a.first(s); i <= a.last(s); ++i) a.code[i] = 2 * s;
}

}  // namespace

const EntDesc* Plan::ent(int kind, int index) const {
  if (index < 0) return nullptr;
  if (kind == 1) return &edges[index];
  if (kind == 2) return &faces[index];
  if (kind == 3) return &blocks[index];
  return nullptr;
}

void Plan::entity_of_cell(int64_t cell, int* kind, int* index) const {
  int c[3];
  int64_t rem = cell;
  int co[3];
  for (int k = 0; k < 3; ++k) {
    c[k] = static_cast<int>(rem % n[k]);
    rem /= n[k];
    co[k] = ax[k].code[c[k]];
  }
  int e = entity_of_key[key_of(co)];
  if (e < 0) {
    *kind = 0;
    *index = -1;
    return;
  }
  *kind = e >> 28;
  *index = e & ((1 << 28) - 1);
}

std::string Plan::build(int dim_, const int n_[3], const int r_[3]) {
  char msg[256];
  if (dim_ != 2 && dim_ != 3) return "dim must be 2 or 3";
  dim = dim_;
  for (int k = 0; k < 3; ++k) {
    bool active = k < dim;
    n[k] = active ? n_[k] : 1;
    r[k] = active ? r_[k] : 1;
    if (active && (n[k] < 2 || n[k] > (1 << 15))) {
      std::snprintf(msg, sizeof msg, "n[%d]=%d out of range [2, 32768]", k, n[k]);
      return msg;
    }
    if (active && (r[k] < 3 || r[k] > 16)) {
      std::snprintf(msg, sizeof msg, "r[%d]=%d out of the supported range [3, 16]", k, r[k]);
      return msg;
    }
    make_axis(ax[k], n[k], r[k]);
    ax[k].active = active;
    ncv[k] = ax[k].nc;
    keydim[k] = 2 * ax[k].nc + 1;
    for (int s = 1; s < ax[k].nc; ++s)
      if (ax[k].empty(s)) return "degenerate geometry: empty bounded segment";
  }
  ncell = int64_t(n[0]) * n[1] * n[2];
  if (ncell > (int64_t(1) << 30)) return "grid too large";
  ncoarse = int64_t(ncv[0]) * ncv[1] * ncv[2];
  stride[0] = 1;
  stride[1] = n[0];
  stride[2] = n[0] * n[1];
  vstride[0] = 1;
  vstride[1] = ncv[0];
  vstride[2] = ncv[0] * ncv[1];

  // ---- entities ---------------------------------------------------------
  entity_of_key.assign(size_t(keydim[0]) * keydim[1] * keydim[2], -1);
  edges.clear();
  faces.clear();
  blocks.clear();
  for (int cz = 0; cz < keydim[2]; ++cz)
    for (int cy = 0; cy < keydim[1]; ++cy)
      for (int cx = 0; cx < keydim[0]; ++cx) {
        int code[3] = {cx, cy, cz};
        EntDesc e{};
        int nopen = 0;
        bool skip = false;
        int choices[3][2];
        int nchoice[3];
        for (int k = 0; k < 3; ++k) {
          const Axis& a = ax[k];
          if (code[k] & 1) {  // plane
            int I = code[k] >> 1;
            e.clo[k] = e.ulo[k] = a.v[I];
            e.cext[k] = e.uext[k] = 1;
            choices[k][0] = I;
            nchoice[k] = 1;
          } else {
            int s = code[k] >> 1;
            if (a.empty(s)) {
              skip = true;
              break;
            }
            ++nopen;
            e.open_mask |= 1 << k;
            e.clo[k] = a.clo(s);
            e.cext[k] = a.chi(s) - a.clo(s) + 1;
            e.ulo[k] = a.first(s);
            e.uext[k] = a.last(s) - a.first(s) + 1;
            if (a.bounded(s)) {
              e.bounded_mask |= 1 << k;
              choices[k][0] = s - 1;
              choices[k][1] = s;
              nchoice[k] = 2;
            } else {
              choices[k][0] = (s == 0) ? 0 : a.nc - 1;
              nchoice[k] = 1;
            }
          }
        }
        if (skip || nopen == 0) continue;
        e.nu = e.uext[0] * e.uext[1] * e.uext[2];
        // corners in ascending vertex id: axis 0 bit fastest
        e.nc = 0;
        e.cbits = 0;
        for (int bz = 0; bz < nchoice[2]; ++bz)
          for (int by = 0; by < nchoice[1]; ++by)
            for (int bx = 0; bx < nchoice[0]; ++bx) {
              int I[3] = {choices[0][bx], choices[1][by], choices[2][bz]};
              int b[3] = {bx, by, bz};
              e.vid[e.nc] = I[0] * vstride[0] + I[1] * vstride[1] + I[2] * vstride[2];
              int bits = 0;
              for (int k = 0; k < 3; ++k)
                if (nchoice[k] == 2 && b[k] == 1) bits |= 1 << k;
              e.cbits |= bits << (3 * e.nc);
              ++e.nc;
            }
        for (int i = e.nc; i < kMaxCorners; ++i) e.vid[i] = -1;
        for (int i = 0; i < 6; ++i) e.side_ent[i] = -1, e.side_slot[i] = -1;
        e.inbase = -1;
        e.nslot = 0;
        e.eptr0 = e.eptr1 = 0;
        int key = key_of(code);
        std::vector<EntDesc>* list = nopen == 1 ? &edges : nopen == 2 ? &faces : &blocks;
        entity_of_key[key] = (nopen << 28) | int(list->size());
        list->push_back(e);
      }

  // ---- routing of adjoint loads: blocks -> faces, faces -> edges ----------
  auto lookup = [&](const int code[3], int want_kind) -> int {
    int e = entity_of_key[key_of(code)];
    if (e < 0 || (e >> 28) != want_kind) return -1;
    return e & ((1 << 28) - 1);
  };
  auto item_codes = [&](const EntDesc& e, int code[3]) {
    for (int k = 0; k < 3; ++k) code[k] = ax[k].code[e.ulo[k]];
  };
  for (auto& b : blocks) {
    int code[3];
    item_codes(b, code);
    for (int k = 0; k < 3; ++k) {
      int s = code[k] >> 1;
      const Axis& a = ax[k];
      // lower side: the plane below the segment; the block is above it (slot 1)
      if (s > 0) {
        int c2[3] = {code[0], code[1], code[2]};
        c2[k] = 2 * (s - 1) + 1;
        b.side_ent[2 * k] = lookup(c2, 2);
        b.side_slot[2 * k] = 1;
      }
      // upper side: the plane above the segment; the block is below it (slot 0)
      if (s < a.nc) {
        int c2[3] = {code[0], code[1], code[2]};
        c2[k] = 2 * s + 1;
        b.side_ent[2 * k + 1] = lookup(c2, 2);
        b.side_slot[2 * k + 1] = 0;
      }
    }
  }
  for (auto& f : faces) {
    int code[3];
    item_codes(f, code);
    int plane_axes[3], np = 0;
    for (int k = 0; k < 3; ++k)
      if (!(f.open_mask >> k & 1)) plane_axes[np++] = k;
    for (int a = 0; a < 3; ++a) {
      if (!(f.open_mask >> a & 1)) continue;
      int s = code[a] >> 1;
      // the receiving edge has planes on axis a and on the face's plane axis
      int rank = 0;
      for (int q = 0; q < np; ++q)
        if (plane_axes[q] < a) ++rank;
      if (s > 0) {
        int c2[3] = {code[0], code[1], code[2]};
        c2[a] = 2 * (s - 1) + 1;
        f.side_ent[2 * a] = lookup(c2, 1);
        f.side_slot[2 * a] = 2 * rank + 1;
      }
      if (s < ax[a].nc) {
        int c2[3] = {code[0], code[1], code[2]};
        c2[a] = 2 * s + 1;
        f.side_ent[2 * a + 1] = lookup(c2, 1);
        f.side_slot[2 * a + 1] = 2 * rank + 0;
      }
    }
  }
  // incoming-load buffers: faces receive from 2 blocks (3-D only), edges from 4 faces
  inbuf_size = 0;
  if (dim == 3)
    for (auto& f : faces) {
      f.nslot = 2;
      f.inbase = int(inbuf_size);
      inbuf_size += int64_t(2) * f.nc * f.nu;
    }
  for (auto& e : edges) {
    e.nslot = 4;
    e.inbase = int(inbuf_size);
    inbuf_size += int64_t(4) * e.nc * e.nu;
  }
  if (inbuf_size > (int64_t(1) << 31) - 1) return "adjoint load buffer too large";

  // ---- energy blocks and the coarse operator pattern ------------------------
  kent_size = 0;
  max_closure = 0;
  max_nu_edge = max_nu_face = max_nu_block = 0;
  std::vector<std::pair<int64_t, int>> contrib;
  auto add_energy = [&](std::vector<EntDesc>& list, int* max_nu) {
    for (auto& e : list) {
      e.kbase = int(kent_size);
      for (int a = 0; a < e.nc; ++a)
        for (int b = 0; b < e.nc; ++b)
          contrib.emplace_back(int64_t(e.vid[a]) * ncoarse + e.vid[b], int(kent_size) + a * e.nc + b);
      kent_size += e.nc * e.nc;
      max_closure = std::max(max_closure, e.cext[0] * e.cext[1] * e.cext[2]);
      *max_nu = std::max(*max_nu, e.nu);
    }
  };
  add_energy(edges, &max_nu_edge);
  add_energy(faces, &max_nu_face);
  add_energy(blocks, &max_nu_block);
  if (kent_size > (int64_t(1) << 31) - 1) return "energy buffer too large";
  std::sort(contrib.begin(), contrib.end());
  krow.assign(ncoarse + 1, 0);
  kcol.clear();
  kcptr.clear();
  kcidx.clear();
  kcptr.push_back(0);
  for (size_t i = 0; i < contrib.size();) {
    int64_t key = contrib[i].first;
    size_t j = i;
    while (j < contrib.size() && contrib[j].first == key) {
      kcidx.push_back(contrib[j].second);
      ++j;
    }
    int row = int(key / ncoarse), col = int(key % ncoarse);
    krow[row + 1]++;
    kcol.push_back(col);
    kcptr.push_back(int(kcidx.size()));
    i = j;
  }
  for (int64_t i = 0; i < ncoarse; ++i) krow[i + 1] += krow[i];
  kdslot.assign(kcol.size(), 0);
  for (int64_t row = 0; row < ncoarse; ++row)
    for (int e = krow[row]; e < krow[row + 1]; ++e) {
      const int col = kcol[e];
      int o = 0, mul = 1;
      for (int k = 0; k < 3; ++k) {
        const int a = int(row / vstride[k]) % ncv[k], b = (col / vstride[k]) % ncv[k];
        const int d = b - a;
        if (d < -1 || d > 1) return "coarse operator pattern wider than 27 points";
        o += (d + 1) * mul;
        mul *= 3;
      }
      kdslot[e] = int(o * ncoarse + row);
    }

  // lane / column caps of the wave-per-corner local solves
  auto caps_of = [&](const std::vector<EntDesc>& list, Caps* c) {
    for (const auto& e : list) {
      int axa, axb, axc;
      if (e.open_mask == 7) {
        axa = 0, axb = 1, axc = 2;
      } else {
        int o[3], no = 0, pl = 0;
        for (int k = 0; k < 3; ++k) {
          if (e.open_mask >> k & 1)
            o[no++] = k;
          else
            pl = k;
        }
        axa = o[0], axb = o[1], axc = pl;
      }
      const int ua = e.uext[axa], ub = e.uext[axb], L = e.uext[axc];
      c->lane = std::max(c->lane, ua * ub);
      c->col = std::max(c->col, L);
      c->nc = std::max(c->nc, e.nc);
      c->plane = std::max(c->plane, wave_plane(ua, ub) * L);
      c->closure = std::max(c->closure, e.cext[0] * e.cext[1] * e.cext[2]);
    }
  };
  caps_face = Caps();
  caps_block = Caps();
  caps_of(faces, &caps_face);
  caps_of(blocks, &caps_block);

  // ---- structure of S_k -----------------------------------------------------
  prow.assign(ncell + 1, 0);
  auto for_cells = [&](const EntDesc& e, auto&& fn) {
    for (int z = 0; z < e.uext[2]; ++z)
      for (int y = 0; y < e.uext[1]; ++y)
        for (int x = 0; x < e.uext[0]; ++x)
          fn(int64_t(e.ulo[0] + x) + int64_t(e.ulo[1] + y) * stride[1] +
             int64_t(e.ulo[2] + z) * stride[2]);
  };
  for (int K = 0; K < ncv[2]; ++K)
    for (int J = 0; J < ncv[1]; ++J)
      for (int I = 0; I < ncv[0]; ++I)
        prow[1 + ax[0].v[I] + int64_t(ax[1].v[J]) * stride[1] + int64_t(ax[2].v[K]) * stride[2]] = 1;
  for (auto* list : {&edges, &faces, &blocks})
    for (auto& e : *list) for_cells(e, [&](int64_t c) { prow[c + 1] = e.nc; });
  for (int64_t i = 0; i < ncell; ++i) {
    int64_t next = int64_t(prow[i]) + prow[i + 1];
    if (next > (int64_t(1) << 31) - 1) return "nnz of the basis exceeds int32";
    prow[i + 1] = int(next);
  }
  pcol.assign(prow[ncell], -1);
  for (int K = 0; K < ncv[2]; ++K)
    for (int J = 0; J < ncv[1]; ++J)
      for (int I = 0; I < ncv[0]; ++I) {
        int64_t c = ax[0].v[I] + int64_t(ax[1].v[J]) * stride[1] + int64_t(ax[2].v[K]) * stride[2];
        pcol[prow[c]] = I * vstride[0] + J * vstride[1] + K * vstride[2];
      }
  for (auto* list : {&edges, &faces, &blocks})
    for (auto& e : *list)
      for_cells(e, [&](int64_t c) {
        for (int a = 0; a < e.nc; ++a) pcol[prow[c] + a] = e.vid[a];
      });
  return std::string();
}

}  // namespace msfv
