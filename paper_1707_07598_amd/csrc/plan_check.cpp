// Host-only consistency check of the plan (plan.cpp), meant to run under
// AddressSanitizer and UndefinedBehaviorSanitizer on the CPU: builds the plan
// of many grids (2-D and 3-D, coarsening 3..16, truncated last coarse cells,
// empty strips) and checks the invariants the kernels rely on.  Prints one
// line per grid; exits non-zero on the first violation.
//
//   g++ -std=c++17 -O1 -g -fsanitize=address,undefined -fno-omit-frame-pointer \
//       plan.cpp plan_check.cpp -o plan_check && ./plan_check
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "plan.hpp"

namespace {

int g_fail = 0;

#define CHECK(cond, ...)                                \
  do {                                                  \
    if (!(cond)) {                                      \
      std::fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
      std::fprintf(stderr, __VA_ARGS__);                \
      std::fprintf(stderr, "\n");                       \
      g_fail = 1;                                       \
      return false;                                     \
    }                                                   \
  } while (0)

bool check_entity(const msfv::Plan& P, const msfv::EntDesc& E, int kind, int idx, std::vector<int>& owner) {
  int nu = 1, opened = 0, bounded = 0;
  for (int k = 0; k < 3; ++k) {
    CHECK(E.clo[k] >= 0 && E.cext[k] >= 1 && E.clo[k] + E.cext[k] <= P.n[k], "closure outside grid");
    CHECK(E.ulo[k] >= E.clo[k] && E.ulo[k] + E.uext[k] <= E.clo[k] + E.cext[k], "own box outside closure");
    nu *= E.uext[k];
    opened += (E.open_mask >> k) & 1;
    bounded += (E.bounded_mask >> k) & 1;
    CHECK(!((E.bounded_mask >> k) & 1) || ((E.open_mask >> k) & 1), "bounded axis not open");
  }
  CHECK(opened == kind, "kind %d has %d open axes", kind, opened);
  CHECK(E.nu == nu && nu >= 1, "own cell count");
  CHECK(E.nc == (1 << bounded) && E.nc <= msfv::kMaxCorners, "corner count");
  for (int c = 0; c < E.nc; ++c) {
    CHECK(E.vid[c] >= 0 && E.vid[c] < P.ncoarse, "corner id out of range");
    CHECK(c == 0 || E.vid[c] > E.vid[c - 1], "corners not ascending");
  }
  CHECK(E.kbase >= 0 && E.kbase + int64_t(E.nc) * E.nc <= P.kent_size, "energy block outside buffer");
  if (E.inbase >= 0)
    CHECK(E.inbase + int64_t(E.nslot) * E.nc * E.nu <= P.inbuf_size, "load slots outside buffer");
  for (int z = 0; z < E.uext[2]; ++z)
    for (int y = 0; y < E.uext[1]; ++y)
      for (int x = 0; x < E.uext[0]; ++x) {
        const int64_t cell = (E.ulo[0] + x) + int64_t(P.stride[1]) * (E.ulo[1] + y) +
                             int64_t(P.stride[2]) * (E.ulo[2] + z);
        CHECK(owner[cell] == -1, "cell owned twice");
        owner[cell] = (kind << 28) | idx;
        CHECK(P.prow[cell + 1] - P.prow[cell] == E.nc, "row length differs from the corner count");
        for (int c = 0; c < E.nc; ++c) CHECK(P.pcol[P.prow[cell] + c] == E.vid[c], "row columns differ");
        int kk = -1, ii = -1;
        P.entity_of_cell(cell, &kk, &ii);
        CHECK(kk == kind && ii == idx, "entity_of_cell disagrees");
      }
  for (int side = 0; side < 6; ++side) {
    const int r = E.side_ent[side];
    if (r < 0) continue;
    const int rk = kind - 1;
    const size_t cnt = rk == 1 ? P.edges.size() : (rk == 2 ? P.faces.size() : 0);
    CHECK(rk >= 1 && size_t(r) < cnt, "side entity out of range");
    const msfv::EntDesc& R = rk == 1 ? P.edges[r] : P.faces[r];
    CHECK(E.side_slot[side] >= 0 && E.side_slot[side] < R.nslot, "side slot out of range");
  }
  return true;
}

bool check(int dim, int nx, int ny, int nz, int rx, int ry, int rz) {
  const int n[3] = {nx, ny, dim == 3 ? nz : 1};
  const int r[3] = {rx, ry, dim == 3 ? rz : 1};
  msfv::Plan P;
  const std::string err = P.build(dim, n, r);
  CHECK(err.empty(), "build failed: %s", err.c_str());
  CHECK(P.ncell == int64_t(n[0]) * n[1] * n[2], "cell count");
  CHECK(int64_t(P.prow.size()) == P.ncell + 1 && P.prow[0] == 0, "row pointer size");
  for (int64_t i = 0; i < P.ncell; ++i) CHECK(P.prow[i + 1] > P.prow[i], "empty or decreasing row");
  CHECK(size_t(P.prow[P.ncell]) == P.pcol.size(), "row pointer end");
  std::vector<int> owner(P.ncell, -1);
  for (int i = 0; i < int(P.edges.size()); ++i)
    if (!check_entity(P, P.edges[i], 1, i, owner)) return false;
  for (int i = 0; i < int(P.faces.size()); ++i)
    if (!check_entity(P, P.faces[i], 2, i, owner)) return false;
  for (int i = 0; i < int(P.blocks.size()); ++i)
    if (!check_entity(P, P.blocks[i], dim, i, owner)) return false;
  int64_t vertices = 0;
  for (int64_t i = 0; i < P.ncell; ++i)
    if (owner[i] == -1) {
      CHECK(P.prow[i + 1] - P.prow[i] == 1, "vertex cell row length");
      CHECK(P.pcol[P.prow[i]] >= 0 && P.pcol[P.prow[i]] < P.ncoarse, "vertex id");
      ++vertices;
    }
  CHECK(vertices == P.ncoarse, "vertex cells %lld != %lld", (long long)vertices, (long long)P.ncoarse);
  // A_k: CSR over vertices, symmetric pattern, diagonal slots in range
  CHECK(int64_t(P.krow.size()) == P.ncoarse + 1, "A_k row pointer size");
  for (int64_t i = 0; i < P.ncoarse; ++i)
    for (int e = P.krow[i]; e < P.krow[i + 1]; ++e) {
      const int j = P.kcol[e];
      CHECK(j >= 0 && j < P.ncoarse, "A_k column out of range");
      bool found = false;
      for (int f = P.krow[j]; f < P.krow[j + 1]; ++f) found |= P.kcol[f] == int(i);
      CHECK(found, "A_k pattern not symmetric");
    }
  CHECK(P.kdslot.size() == P.kcol.size(), "diagonal slot count");
  for (int s : P.kdslot) CHECK(s >= 0 && int64_t(s) < 27 * P.ncoarse, "diagonal slot out of range");
  CHECK(P.kcptr.size() == P.kcol.size() + 1, "energy contributor pointer size");
  for (int e : P.kcidx) CHECK(e >= 0 && e < P.kent_size, "energy contributor out of range");
  std::printf("ok dim=%d n=%dx%dx%d r=%dx%dx%d: %zu edges %zu faces %zu blocks, %lld coarse\n", dim, n[0], n[1],
              n[2], r[0], r[1], r[2], P.edges.size(), P.faces.size(), P.blocks.size(), (long long)P.ncoarse);
  return true;
}

}  // namespace

int main() {
  const int grids[][7] = {
      {3, 13, 11, 9, 4, 4, 4},   {3, 16, 12, 10, 4, 3, 5}, {3, 17, 9, 12, 8, 3, 4}, {3, 18, 10, 7, 5, 3, 3},
      {3, 40, 36, 34, 16, 16, 16}, {3, 4, 4, 4, 4, 4, 4},  {3, 8, 3, 5, 4, 3, 5},   {3, 5, 5, 5, 4, 4, 4},
      {3, 64, 64, 64, 8, 8, 8},  {3, 85, 85, 85, 8, 8, 8}, {3, 47, 33, 29, 16, 8, 4}, {3, 24, 22, 20, 8, 8, 8},
      {2, 32, 32, 1, 4, 4, 1},   {2, 23, 17, 1, 5, 6, 1},  {2, 40, 36, 1, 16, 16, 1}, {2, 9, 7, 1, 4, 3, 1},
      {2, 172, 160, 1, 4, 4, 1}, {3, 31, 29, 27, 3, 3, 3}};
  for (const auto& g : grids)
    if (!check(g[0], g[1], g[2], g[3], g[4], g[5], g[6])) return 1;
  return g_fail;
}
