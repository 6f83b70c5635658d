// Host-side plan of one MSFV problem: coarse vertices, segments, entities,
// the CSR structure of the prolongation S_k and of the coarse operator A_k,
// and the bookkeeping that routes adjoint loads between entities.
//
// The nested coarse partition (Sec. 3.2, step 1) is realised as the
// vertex / dual-block complex of cell-centred MSFV: along every axis the
// coarse vertex I sits at v_I = I*r + floor(min(r, n - I*r)/2); a cell lies
// either on a vertex plane or open in a segment (lower strip, bounded
// segment between two planes, upper strip).  An entity is the tuple of
// per-axis items; its dimension is the number of open axes (edge 1, face 2,
// dual block 3).  Every cell belongs to exactly one entity.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace msfv {

constexpr int kMaxCorners = 8;

// Zero-padded plane buffer of the wave-per-corner local solves, for an own
// box of ua x ub columns: rows of 8 doubles (lane (ia, ib) at row ib + 1,
// entry ia + 1; entry 0 of each row is both its left pad and the previous
// row's right pad) when ua <= 7 and ub <= 8, so each 16-lane quarter of a
// wave reads 16 consecutive doubles; otherwise rows of ua + 2.  Doubles per
// plane (the column axis multiplies it).
constexpr int wave_plane_row(int ua, int ub) { return (ua <= 7 && ub <= 8) ? 8 : ua + 2; }
constexpr int wave_plane(int ua, int ub) { return wave_plane_row(ua, ub) * (ub + 2); }

// Entity descriptor shared by host and device (plain data, 4-byte fields).
struct EntDesc {
  int clo[3];        // closure box: global lower corner
  int cext[3];       // closure box: extents
  int ulo[3];        // own cells (unknowns): global lower corner
  int uext[3];       // own cells: extents (1 on plane axes)
  int open_mask;     // bit k: axis k is open
  int bounded_mask;  // bit k: axis k is open in a bounded segment
  int nc;            // number of corners (2^popcount(bounded_mask))
  int nu;            // number of own cells
  int vid[kMaxCorners];  // corner vertex ids, ascending (= column order of S_k rows)
  int cbits;         // 3 bits per corner: bit k set if the corner is the upper plane on axis k
  int kbase;         // offset of this entity's nc*nc energy block
  int inbase;        // offset of this entity's incoming adjoint loads (-1: none)
  int nslot;         // incoming load slots (faces 2, edges 4, blocks 0)
  int side_ent[6];   // entity (next lower kind) across side 2*k+hi, -1 if none
  int side_slot[6];  // slot of this entity in that receiver
  int eptr0, eptr1;  // electrodes owned by this entity: [eptr0, eptr1)
};

struct Axis {
  int n = 1, r = 1, nc = 1;
  bool active = true;
  std::vector<int> v;  // vertex plane positions
  // segment s in [0, nc]: low strip, bounded (v[s-1], v[s]), high strip
  int first(int s) const { return s == 0 ? 0 : v[s - 1] + 1; }
  int last(int s) const { return s == nc ? n - 1 : v[s] - 1; }
  int clo(int s) const { return s == 0 ? 0 : v[s - 1]; }
  int chi(int s) const { return s == nc ? n - 1 : v[s]; }
  bool bounded(int s) const { return s > 0 && s < nc; }
  bool empty(int s) const { return last(s) < first(s); }
  // item code along the axis: segment s -> 2s, plane I -> 2I+1
  std::vector<int> code;  // per cell
};

struct Plan {
  int dim = 3;
  int n[3] = {1, 1, 1};
  int r[3] = {1, 1, 1};
  Axis ax[3];
  int64_t ncell = 0;
  int ncv[3] = {1, 1, 1};
  int64_t ncoarse = 0;
  int stride[3] = {1, 1, 1};   // cell strides
  int vstride[3] = {1, 1, 1};  // vertex strides

  std::vector<EntDesc> edges, faces, blocks;  // 1, 2, 3 open axes
  std::vector<int> entity_of_key;             // key -> (kind<<28)|index, or -1
  int keydim[3] = {1, 1, 1};

  std::vector<int> prow, pcol;     // S_k CSR structure
  std::vector<int> krow, kcol;     // A_k CSR structure
  std::vector<int> kdslot;         // per A_k nonzero: slot o*ncoarse + row of its diagonal o
  std::vector<int> kcptr, kcidx;   // per A_k nonzero: energy-block entries summed into it
  int64_t kent_size = 0;           // doubles in the energy-block buffer
  int64_t inbuf_size = 0;          // doubles in the adjoint-load buffer
  int max_closure = 0;             // largest closure box (cells)
  int max_nu_face = 0, max_nu_block = 0, max_nu_edge = 0;
  // geometry caps of a launch over faces or blocks (lane plane, column, corners,
  // zero-padded plane buffer); see the wave-per-corner kernels
  struct Caps {
    int lane = 0, col = 0, nc = 0, plane = 0, closure = 0;
  } caps_face, caps_block;

  // Build; returns an empty string on success or an error message.
  std::string build(int dim, const int n[3], const int r[3]);

  int key_of(const int code[3]) const {
    return code[0] + keydim[0] * (code[1] + keydim[1] * code[2]);
  }
  // kind: 0 vertex, 1 edge, 2 face, 3 block; index into the list; -1 if none
  void entity_of_cell(int64_t cell, int* kind, int* index) const;
  const EntDesc* ent(int kind, int index) const;
};

}  // namespace msfv
