// Wave-per-corner local solves for faces and dual blocks whose own cells fit
// a 64-lane plane (coarsening r <= 8).
//
// A workgroup handles one entity E (a face or a dual block).  After a shared
// setup (closure conductivities, two-point transmissibilities and the Jacobi
// scaling d^{-1/2}), wavefront c works on corner c of E alone: the corners
// are independent right-hand sides of the same local matrix, so the
// conjugate-gradient iteration needs no workgroup barrier.  Lane l owns the
// column (ia, ib) of the entity's own-cell box over its two lane axes and
// keeps the column's cells along the third axis in registers; neighbours
// along the lane axes are exchanged through a zero-padded plane buffer in LDS
// (Dirichlet and outside neighbours read 0), neighbours along the column come
// from registers.  CG runs on the symmetrically scaled operator
// D^{-1/2} A D^{-1/2} (Jacobi-PCG on A in exact arithmetic) with two
// wavefront reductions per iteration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "kernels.hpp"

namespace msfv {

namespace {

constexpr int kWave = 64;

__device__ __forceinline__ double harm(double a, double b) { return 2.0 * a * b / (a + b); }
// d/dm_a of harm(a, b) for sigma = exp(m)
__device__ __forceinline__ double dharm(double a, double b) {
  const double s = a + b;
  return 2.0 * a * b * b / (s * s);
}

// DPP lane exchange of a double within 16-lane rows (every lane written).
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}

// v[l] + v[l ^ 16] (ROW32 = false) or v[l] + v[l ^ 32] (ROW32 = true) in every
// lane: the gfx950 row-swap instructions exchange half of two copies of v,
// and the two results hold the partner values in complementary halves.
template <bool ROW32>
__device__ __forceinline__ double swap_add(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  if constexpr (ROW32) {
    const auto a = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto b = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    return __hiloint2double(b[0], a[0]) + __hiloint2double(b[1], a[1]);
  } else {
    const auto a = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto b = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    return __hiloint2double(b[0], a[0]) + __hiloint2double(b[1], a[1]);
  }
}

// Wavefront sum, bitwise identical in every lane (each stage adds the same
// two operands in both partner lanes): exchange within quads (xor 1, xor 2),
// half rows and rows by DPP, then across row pairs and wave halves.
__device__ __forceinline__ double wsum(double v) {
  v += dpp_move<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_move<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_move<0x141>(v);  // row_half_mirror
  v += dpp_move<0x140>(v);  // row_mirror
  v = swap_add<false>(v);
  return swap_add<true>(v);
}

// Block sum of N values per thread in a fixed order: wavefront sums, then
// thread i adds the per-wave partials of value i in wave order.  On return
// red[0..N) holds the sums, visible to every thread.  red holds NWAVE * N
// doubles.
template <int NWAVE, int N>
__device__ __forceinline__ void block_sum(const double (&v)[N], double* red) {
  const int wid = threadIdx.x / 64, lane = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const double t = wsum(v[i]);
    if (lane == 0) red[wid * N + i] = t;
  }
  __syncthreads();
  if (threadIdx.x < N) {
    double t = red[threadIdx.x];
    for (int q = 1; q < NWAVE; ++q) t += red[q * N + threadIdx.x];
    red[threadIdx.x] = t;  // only this thread touches column threadIdx.x
  }
  __syncthreads();
}

// a / b for the CG step lengths.  Short columns (faces) use the hardware
// reciprocal refined by one Newton step (a few ulp; the iteration only needs
// the ratio, not its rounding), which measured faster there; long columns
// keep the full division, which measured faster in the dual-block loop.
template <int LMAX>
__device__ __forceinline__ double step_div(double a, double b) {
  if constexpr (LMAX <= 3) {
    const double r0 = __builtin_amdgcn_rcp(b);
    const double e = fma(-b, r0, 1.0);
    return a * fma(r0, e, r0);
  } else {
    return a / b;
  }
}

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ double p_lookup(const int* __restrict__ prow, const int* __restrict__ pcol,
                                           const double* __restrict__ pval, int gid, int vid) {
  const int a = prow[gid], b = prow[gid + 1];
  double v = 0.0;
  for (int e = a; e < b; ++e)
    if (pcol[e] == vid) v = pval[e];
  return v;
}

__device__ __forceinline__ int sel3(int k, int a0, int a1, int a2) {
  return k == 0 ? a0 : (k == 1 ? a1 : a2);
}

// Lane / column geometry of an entity: lane axes a, b and column axis c, with
// strides of each in own-cell index space (u), global cell space (g) and
// closure space (s).
struct WGeo {
  int axa, axb, axc;
  int Ua, Ub, L;
  int ua, ub, uc;  // own-index strides
  int ga, gb, gc;  // global strides
  int sa, sb, sc;  // closure strides
  int lw;          // lanes a row of the lane plane (lane = ia + lw * ib)
  int pa, plane;   // padded row length and padded plane size
  int g0, s0;      // global id and closure index of the own-box origin
};

__device__ __forceinline__ WGeo wave_geo(const EntDesc& E, const GridInfo& g) {
  WGeo w;
  if (E.open_mask == 7) {
    w.axa = 0;
    w.axb = 1;
    w.axc = 2;
  } else {
    // the two open axes are the lane axes; the plane axis is the column
    w.axc = (E.open_mask & 1) == 0 ? 0 : ((E.open_mask & 2) == 0 ? 1 : 2);
    w.axa = w.axc == 0 ? 1 : 0;
    w.axb = w.axc == 2 ? 1 : 2;
  }
  const int us1 = E.uext[0], us2 = E.uext[0] * E.uext[1];
  const int cs1 = E.cext[0], cs2 = E.cext[0] * E.cext[1];
  w.Ua = sel3(w.axa, E.uext[0], E.uext[1], E.uext[2]);
  w.Ub = sel3(w.axb, E.uext[0], E.uext[1], E.uext[2]);
  w.L = sel3(w.axc, E.uext[0], E.uext[1], E.uext[2]);
  w.ua = sel3(w.axa, 1, us1, us2);
  w.ub = sel3(w.axb, 1, us1, us2);
  w.uc = sel3(w.axc, 1, us1, us2);
  w.ga = sel3(w.axa, 1, g.s1, g.s2);
  w.gb = sel3(w.axb, 1, g.s1, g.s2);
  w.gc = sel3(w.axc, 1, g.s1, g.s2);
  w.sa = sel3(w.axa, 1, cs1, cs2);
  w.sb = sel3(w.axb, 1, cs1, cs2);
  w.sc = sel3(w.axc, 1, cs1, cs2);
  // rows of 8 lanes and 8 doubles where the box allows: a 16-lane quarter
  // of the wave then touches 16 consecutive doubles of the plane buffer
  w.pa = wave_plane_row(w.Ua, w.Ub);
  w.lw = w.pa == 8 ? 8 : w.Ua;
  w.plane = wave_plane(w.Ua, w.Ub);
  w.g0 = E.ulo[0] + g.s1 * E.ulo[1] + g.s2 * E.ulo[2];
  w.s0 = (E.ulo[0] - E.clo[0]) + cs1 * (E.ulo[1] - E.clo[1]) + cs2 * (E.ulo[2] - E.clo[2]);
  return w;
}

// Neighbour classes of the cell at lane position (ia, ib) and column index k:
// bit d = 2*axis + plus of fm: the reduced operator has that flux; of um:
// the neighbour is an own cell.
__device__ __forceinline__ void cell_masks(const EntDesc& E, const WGeo& w, int ia, int ib, int k,
                                           int* fm, int* um) {
  int f = 0, u = 0;
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    if (!((E.open_mask >> ax) & 1)) continue;
    const int own = ax == w.axa ? ia : (ax == w.axb ? ib : k);
    const int ext = sel3(ax, E.uext[0], E.uext[1], E.uext[2]);
    const int off = sel3(ax, E.ulo[0] - E.clo[0], E.ulo[1] - E.clo[1], E.ulo[2] - E.clo[2]);
    const int cext = sel3(ax, E.cext[0], E.cext[1], E.cext[2]);
    const int cl = own + off;
    if (cl - 1 >= 0) f |= 1 << (2 * ax);
    if (cl + 1 < cext) f |= 1 << (2 * ax + 1);
    if (own - 1 >= 0) u |= 1 << (2 * ax);
    if (own + 1 < ext) u |= 1 << (2 * ax + 1);
  }
  *fm = f;
  *um = u & f;
}

// The fine fluxes an entity owns as a flat list that a workgroup strides
// through in step: for each open axis k, the +k flux of every own cell (to
// an own cell, or on the upper face to a closure cell), then the -k flux of
// the own cells on the lower face (to a closure cell).  Consecutive items
// share a direction, so the lanes of a wave take the same branch; a flux
// that would leave the closure (the domain boundary) comes back invalid.
struct OwnedFlux {
  int u, ci, gid;  // own cell: own index, closure index, global id
  int ax, sgn;     // direction of the flux from the own cell
  bool own;        // the neighbour is an own cell
  bool valid;
};

__device__ __forceinline__ int owned_flux_count(const EntDesc& E) {
  int n = 0;
#pragma unroll
  for (int k = 0; k < 3; ++k)
    if ((E.open_mask >> k) & 1) n += E.nu + E.nu / sel3(k, E.uext[0], E.uext[1], E.uext[2]);
  return n;
}

__device__ __forceinline__ OwnedFlux owned_flux(const EntDesc& E, const GridInfo& g, int g0, int item) {
  OwnedFlux f;
  f.valid = false;
  const int e0 = E.uext[0], e1 = E.uext[1], e2 = E.uext[2];
  int ax = -1, sgn = 1, idx = item;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (ax >= 0 || !((E.open_mask >> k) & 1)) continue;
    const int face = E.nu / sel3(k, e0, e1, e2);
    if (idx < E.nu) {
      ax = k;
      sgn = 1;
    } else if (idx < E.nu + face) {
      ax = k;
      sgn = -1;
      idx -= E.nu;
    } else {
      idx -= E.nu + face;
    }
  }
  if (ax < 0) return f;
  int ux, uy, uz;
  if (sgn > 0) {
    ux = idx % e0;
    const int t = idx / e0;
    uy = t % e1;
    uz = t / e1;
  } else if (ax == 0) {
    ux = 0;
    uy = idx % e1;
    uz = idx / e1;
  } else if (ax == 1) {
    ux = idx % e0;
    uy = 0;
    uz = idx / e0;
  } else {
    ux = idx % e0;
    uy = idx / e0;
    uz = 0;
  }
  const int o0 = E.ulo[0] - E.clo[0], o1 = E.ulo[1] - E.clo[1], o2 = E.ulo[2] - E.clo[2];
  const int own = sel3(ax, ux, uy, uz);
  const int cl = own + sel3(ax, o0, o1, o2);
  const int cext = sel3(ax, E.cext[0], E.cext[1], E.cext[2]);
  f.valid = sgn > 0 ? cl + 1 < cext : cl - 1 >= 0;
  f.own = sgn > 0 && own + 1 < sel3(ax, e0, e1, e2);
  f.u = ux + e0 * (uy + e1 * uz);
  f.ci = (ux + o0) + E.cext[0] * ((uy + o1) + E.cext[1] * (uz + o2));
  f.gid = g0 + ux + g.s1 * uy + g.s2 * uz;
  f.ax = ax;
  f.sgn = sgn;
  return f;
}

// Natural strides of global axis k in own-cell index space, closure space
// and global cell space (k is a compile-time constant after unrolling).
__device__ __forceinline__ int ustr(const EntDesc& E, int k) {
  return k == 0 ? 1 : (k == 1 ? E.uext[0] : E.uext[0] * E.uext[1]);
}
__device__ __forceinline__ int cstr(const EntDesc& E, int k) {
  return k == 0 ? 1 : (k == 1 ? E.cext[0] : E.cext[0] * E.cext[1]);
}
__device__ __forceinline__ int gstr(const GridInfo& g, int k) {
  return k == 0 ? 1 : (k == 1 ? g.s1 : g.s2);
}

// global coordinates of the cell at lane position (ia, ib), column index k
__device__ __forceinline__ void own_coords(const EntDesc& E, const WGeo& w, int ia, int ib, int k,
                                           int gc[3]) {
#pragma unroll
  for (int ax = 0; ax < 3; ++ax)
    gc[ax] = sel3(ax, E.ulo[0], E.ulo[1], E.ulo[2]) + (ax == w.axa ? ia : (ax == w.axb ? ib : k));
}

// sigma on the closure, sqrt of the operator diagonal, scaled transmissibilities
template <int BLOCK>
__device__ void shared_setup(const EntDesc& E, const GridInfo& g, const double* __restrict__ sigma,
                             double* sig, double* dsq, double* tt, const WGeo& w, bool op = true) {
  // sigma = exp(m) of the call's model, formed once per cell by the model copy
  const int ncl = E.cext[0] * E.cext[1] * E.cext[2];
  for (int i = threadIdx.x; i < ncl; i += BLOCK) {
    const int lx = i % E.cext[0];
    const int t = i / E.cext[0];
    const int ly = t % E.cext[1];
    const int lz = t / E.cext[1];
    sig[i] = sigma[(E.clo[0] + lx) + g.s1 * (E.clo[1] + ly) + g.s2 * (E.clo[2] + lz)];
  }
  __syncthreads();
  if (!op) return;  // sigma only: no local solve follows
  const int ncol = w.Ua * w.Ub;
  for (int i = threadIdx.x; i < ncol * w.L; i += BLOCK) {
    const int col = i % ncol, k = i / ncol;
    const int ia = col % w.Ua, ib = col / w.Ua;
    int fm, um;
    cell_masks(E, w, ia, ib, k, &fm, &um);
    const int ci = w.s0 + ia * w.sa + ib * w.sb + k * w.sc;
    double d = 0.0;
#pragma unroll
    for (int dd = 0; dd < 6; ++dd)
      if ((fm >> dd) & 1) {
        const int st = cstr(E, dd >> 1);
        d += harm(sig[ci], sig[ci + ((dd & 1) ? st : -st)]);
      }
    dsq[ia * w.ua + ib * w.ub + k * w.uc] = sqrt(d);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < ncol * w.L; i += BLOCK) {
    const int col = i % ncol, k = i / ncol;
    const int ia = col % w.Ua, ib = col / w.Ua;
    int fm, um;
    cell_masks(E, w, ia, ib, k, &fm, &um);
    const int ci = w.s0 + ia * w.sa + ib * w.sb + k * w.sc;
    const int u = ia * w.ua + ib * w.ub + k * w.uc;
#pragma unroll
    for (int dd = 0; dd < 6; ++dd) {
      double v = 0.0;
      if ((um >> dd) & 1) {
        const int sgn = (dd & 1) ? 1 : -1;
        v = harm(sig[ci], sig[ci + sgn * cstr(E, dd >> 1)]) /
            (dsq[u] * dsq[u + sgn * ustr(E, dd >> 1)]);
      }
      tt[dd * E.nu + u] = v;
    }
  }
}

// One lane's column of scaled transmissibilities along the lane axes and the column.
template <int LMAX>
struct Column {
  double tz[LMAX], tam[LMAX], tap[LMAX], tbm[LMAX], tbp[LMAX];
};

template <int LMAX>
__device__ __forceinline__ void load_column(const EntDesc& E, const WGeo& w, bool valid, int ia, int ib,
                                            const double* tt, Column<LMAX>& C) {
#pragma unroll
  for (int k = 0; k < LMAX; ++k) {
    C.tz[k] = C.tam[k] = C.tap[k] = C.tbm[k] = C.tbp[k] = 0.0;
    if (!valid || k >= w.L) continue;
    const int u = ia * w.ua + ib * w.ub + k * w.uc;
    C.tam[k] = tt[(2 * w.axa) * E.nu + u];
    C.tap[k] = tt[(2 * w.axa + 1) * E.nu + u];
    C.tbm[k] = tt[(2 * w.axb) * E.nu + u];
    C.tbp[k] = tt[(2 * w.axb + 1) * E.nu + u];
    C.tz[k] = tt[(2 * w.axc + 1) * E.nu + u];
  }
}

// Conjugate gradients on the scaled operator for one corner, run by one
// wavefront.  y holds the scaled right-hand side on entry and the scaled
// solution on exit.  pbuf: this wave's padded plane buffer.
// With a start vector (x0 != nullptr, the scaled initial guess), the
// iteration starts from r = y - A x0 and the stop test stays relative to the
// right-hand side y, as without one.
template <int LMAX>
__device__ int wave_cg(const WGeo& w, bool valid, int ia, int ib, const Column<LMAX>& C,
                       double (&y)[LMAX], double* pbuf, double tol2, int maxit, bool* ok,
                       const double (*x0)[LMAX] = nullptr, double* res2 = nullptr) {
  const int lane = threadIdx.x & (kWave - 1);
  for (int i = lane; i < w.plane * w.L; i += kWave) pbuf[i] = 0.0;
  wave_sync_lds();
  const int pidx = (ib + 1) * w.pa + (ia + 1);
  const int pidx_safe = valid ? pidx : w.pa + 1;
  double r[LMAX], p[LMAX];
  double rr = 0.0;
#pragma unroll
  for (int k = 0; k < LMAX; ++k) {
    r[k] = y[k];
    p[k] = y[k];
    y[k] = 0.0;
    rr += r[k] * r[k];
  }
  rr = wsum(rr);
  const double bb = rr;
  int it = 0;
  *ok = true;
  if (res2) *res2 = 0.0;
  if (!(bb > 0.0)) return 0;
  if (x0) {
    // r = y - A x0 (the in-plane neighbours of x0 through the plane buffer)
    if (valid) {
#pragma unroll
      for (int k = 0; k < LMAX; ++k)
        if (k < w.L) pbuf[k * w.plane + pidx] = (*x0)[k];
    }
    wave_sync_lds();
    rr = 0.0;
#pragma unroll
    for (int k = 0; k < LMAX; ++k) {
      double s = (*x0)[k];
      if (k > 0) s -= C.tz[k - 1] * (*x0)[k - 1];
      if (k + 1 < LMAX) s -= C.tz[k] * (*x0)[k + 1];
      const double* pl = pbuf + min(k, w.L - 1) * w.plane + pidx_safe;
      s -= C.tam[k] * pl[-1] + C.tap[k] * pl[1] + C.tbm[k] * pl[-w.pa] + C.tbp[k] * pl[w.pa];
      r[k] -= s;
      p[k] = r[k];
      y[k] = (*x0)[k];
      rr += r[k] * r[k];
    }
    rr = wsum(rr);
    wave_sync_lds();  // all lanes finished reading x0 before the loop writes p
    if (rr <= tol2 * bb) {
      if (res2) *res2 = rr / bb;
      return 0;
    }
  }
  double last = rr;  // r.r of the current iterate
  while (true) {
    if (it >= maxit) {
      *ok = false;
      break;
    }
    ++it;
    if (valid) {
#pragma unroll
      for (int k = 0; k < LMAX; ++k)
        if (k < w.L) pbuf[k * w.plane + pidx] = p[k];
    }
    wave_sync_lds();
    // In-plane neighbours from LDS.  The loads are unconditional so that all
    // of them issue back to back: lanes outside the plane read an interior
    // position and planes past the column read the last one, both with zero
    // coefficients (zero-initialised buffer, finite values).
    double q[LMAX];
    double pq = 0.0;
#pragma unroll
    for (int k = 0; k < LMAX; ++k) {
      double s = p[k];
      if (k > 0) s -= C.tz[k - 1] * p[k - 1];
      if (k + 1 < LMAX) s -= C.tz[k] * p[k + 1];
      const double* pl = pbuf + min(k, w.L - 1) * w.plane + pidx_safe;
      s -= C.tam[k] * pl[-1] + C.tap[k] * pl[1] + C.tbm[k] * pl[-w.pa] + C.tbp[k] * pl[w.pa];
      q[k] = s;
      pq += p[k] * s;
    }
    pq = wsum(pq);
    const double alpha = pq != 0.0 ? step_div<LMAX>(rr, pq) : 0.0;
    double rn = 0.0;
#pragma unroll
    for (int k = 0; k < LMAX; ++k) {
      y[k] += alpha * p[k];
      r[k] -= alpha * q[k];
      rn += r[k] * r[k];
    }
    rn = wsum(rn);
    last = rn;
    if (rn <= tol2 * bb) break;
    if (rn != rn) {
      *ok = false;
      break;
    }
    const double beta = step_div<LMAX>(rn, rr);
    rr = rn;
#pragma unroll
    for (int k = 0; k < LMAX; ++k) p[k] = r[k] + beta * p[k];
    wave_sync_lds();  // all lanes finished reading the previous directions
  }
  if (res2) *res2 = last / bb;
  return it;
}

// Four wavefront sums at once, every lane receiving all four totals.
// Reduce-scatter: swapping wave halves leaves the half sums of values 0 and
// 2 (1 and 3) in the low and high halves of one register; swapping odd and
// even rows then leaves value q's partial in row q; DPP finishes each row,
// and row q's total is read from lane 16 q.  About a third of the
// instructions of four separate sums, bitwise deterministic.
__device__ __forceinline__ void reduce4(double (&v)[4]) {
  auto swap32_add = [](double x, double y) {
    const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(x), __double2loint(y), false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(x), __double2hiint(y), false, false);
    return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
  };
  auto swap16_add = [](double x, double y) {
    const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(x), __double2loint(y), false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(x), __double2hiint(y), false, false);
    return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
  };
  // lanes 0-31: value 0 (1), lanes 32-63: value 2 (3), each over the two halves
  const double s02 = swap32_add(v[0], v[2]);
  const double s13 = swap32_add(v[1], v[3]);
  // row q (lanes 16q .. 16q + 15): value q over the four rows
  double t = swap16_add(s02, s13);
  t += dpp_move<0xB1>(t);   // quad_perm [1,0,3,2]
  t += dpp_move<0x4E>(t);   // quad_perm [2,3,0,1]
  t += dpp_move<0x141>(t);  // row_half_mirror
  t += dpp_move<0x140>(t);  // row_mirror
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(t), 16 * q);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(t), 16 * q);
    v[q] = __hiloint2double(hi, lo);
  }
}

// Conjugate gradients for the (up to) four corners of an entity in lockstep,
// run by one wavefront: the corners share the operator columns and the loop,
// and their wave sums go through reduce4.  buf holds four padded plane
// buffers of plane_cap doubles.  A corner that has converged (or has a zero
// load) takes zero steps while the others iterate; its[c] and ok[c] report
// each corner.
template <int LMAX>
__device__ void wave_cg4(const WGeo& w, bool valid, int ia, int ib, const Column<LMAX>& C,
                         double (&y)[4][LMAX], double* buf, int plane_cap, double tol2, int maxit,
                         int (&its)[4], bool (&ok)[4], const double (*x0)[4][LMAX] = nullptr,
                         double* res2 = nullptr) {
  const int lane = threadIdx.x & (kWave - 1);
  for (int i = lane; i < 4 * plane_cap; i += kWave) buf[i] = 0.0;
  wave_sync_lds();
  const int pidx = (ib + 1) * w.pa + (ia + 1);
  const int pidx_safe = valid ? pidx : w.pa + 1;
  double r[4][LMAX], p[4][LMAX], rr[4], bb[4];
  bool done[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    rr[c] = 0.0;
#pragma unroll
    for (int k = 0; k < LMAX; ++k) {
      r[c][k] = p[c][k] = y[c][k];
      y[c][k] = 0.0;
      rr[c] += r[c][k] * r[c][k];
    }
  }
  reduce4(rr);
  double last[4];  // r.r of each corner's current iterate
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    bb[c] = rr[c];
    last[c] = rr[c];
    done[c] = !(bb[c] > 0.0);
    its[c] = 0;
    ok[c] = true;
  }
  if (x0) {
    // start vectors (a corner with a zero right-hand side keeps a zero
    // start): r = y - A x0, the stop test still relative to y
    if (valid) {
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int k = 0; k < LMAX; ++k)
          if (k < w.L) buf[c * plane_cap + k * w.plane + pidx] = done[c] ? 0.0 : (*x0)[c][k];
    }
    wave_sync_lds();
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      rr[c] = 0.0;
      if (done[c]) continue;
#pragma unroll
      for (int k = 0; k < LMAX; ++k) {
        double s = (*x0)[c][k];
        if (k > 0) s -= C.tz[k - 1] * (*x0)[c][k - 1];
        if (k + 1 < LMAX) s -= C.tz[k] * (*x0)[c][k + 1];
        const double* pl = buf + c * plane_cap + min(k, w.L - 1) * w.plane + pidx_safe;
        s -= C.tam[k] * pl[-1] + C.tap[k] * pl[1] + C.tbm[k] * pl[-w.pa] + C.tbp[k] * pl[w.pa];
        r[c][k] -= s;
        p[c][k] = r[c][k];
        y[c][k] = (*x0)[c][k];
        rr[c] += r[c][k] * r[c][k];
      }
    }
    reduce4(rr);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      last[c] = rr[c];
      if (!done[c] && rr[c] <= tol2 * bb[c]) {
        done[c] = true;
#pragma unroll
        for (int k = 0; k < LMAX; ++k) p[c][k] = 0.0;
      }
    }
    wave_sync_lds();  // all lanes finished reading the start vectors
  }
  int it = 0;
  while (!(done[0] && done[1] && done[2] && done[3])) {
    if (it >= maxit) {
#pragma unroll
      for (int c = 0; c < 4; ++c)
        if (!done[c]) ok[c] = false, its[c] = it;
      break;
    }
    ++it;
    if (valid) {
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int k = 0; k < LMAX; ++k)
          if (k < w.L) buf[c * plane_cap + k * w.plane + pidx] = p[c][k];
    }
    wave_sync_lds();
    double q[4][LMAX], pq[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      pq[c] = 0.0;
#pragma unroll
      for (int k = 0; k < LMAX; ++k) {
        double s = p[c][k];
        if (k > 0) s -= C.tz[k - 1] * p[c][k - 1];
        if (k + 1 < LMAX) s -= C.tz[k] * p[c][k + 1];
        const double* pl = buf + c * plane_cap + min(k, w.L - 1) * w.plane + pidx_safe;
        s -= C.tam[k] * pl[-1] + C.tap[k] * pl[1] + C.tbm[k] * pl[-w.pa] + C.tbp[k] * pl[w.pa];
        q[c][k] = s;
        pq[c] += p[c][k] * s;
      }
    }
    reduce4(pq);
    double rn[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const double al = (done[c] || pq[c] == 0.0) ? 0.0 : step_div<LMAX>(rr[c], pq[c]);
      rn[c] = 0.0;
#pragma unroll
      for (int k = 0; k < LMAX; ++k) {
        y[c][k] += al * p[c][k];
        r[c][k] -= al * q[c][k];
        rn[c] += r[c][k] * r[c][k];
      }
    }
    reduce4(rn);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      last[c] = rn[c];
      double be = 0.0;
      if (!done[c]) {
        if (rn[c] <= tol2 * bb[c]) {
          done[c] = true;
          its[c] = it;
        } else if (rn[c] != rn[c]) {
          done[c] = true;
          ok[c] = false;
          its[c] = it;
        } else {
          be = step_div<LMAX>(rn[c], rr[c]);
          rr[c] = rn[c];
        }
      }
      // a finished corner keeps a zero direction: zero steps, finite products
#pragma unroll
      for (int k = 0; k < LMAX; ++k) p[c][k] = done[c] ? 0.0 : r[c][k] + be * p[c][k];
    }
    wave_sync_lds();  // all lanes finished reading the previous directions
  }
  if (res2) {
    double m2 = 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (bb[c] > 0.0) {
        double q = last[c] / bb[c];
        if (!(q >= 0.0)) q = __builtin_huge_val();
        m2 = fmax(m2, q);
      }
    *res2 = m2;
  }
}

__device__ __forceinline__ double lagrange_value(const EntDesc& E, const int gc[3], int ci) {
  double v = 1.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (!((E.bounded_mask >> k) & 1)) continue;
    const double lo = E.clo[k], hi = E.clo[k] + E.cext[k] - 1;
    const double x = gc[k];
    const bool upper = (E.cbits >> (3 * ci + k)) & 1;
    v *= upper ? (x - lo) / (hi - lo) : (hi - x) / (hi - lo);
  }
  return v;
}

struct WaveLds {
  double* sig;
  double* phi;   // basis values of the corners on the closure: phi[c*ncl + i]
  double* dsq;
  double* tt;    // 6 * nu (aliases pbuf)
  double* pbuf;  // NWAVE * plane_cap
  double* Mm;
  double* Sm;
  int* wit;      // per corner: CG iterations
  int* sbase;    // adjoint: per side d and corner c, offset of the receiver's load slot (-1: none)
  int* sgeo;     // adjoint: per side, receiver-local index = gx + gy*s1 + gz*s2 + off: {s1, s2, off}
  double* red;   // block reductions (RED waves x 36 values)
};

// LDS layout: sig, the basis table of PHIC corners, dsq, small tables, the
// block-reduction scratch of RED waves, then the shared plane-buffer region.
template <int NWAVE, int PHIC = 8, int RED = 8>
__device__ __forceinline__ WaveLds carve(const LocalParams& a, double* lds) {
  WaveLds L;
  L.sig = lds;
  L.phi = L.sig + a.sig_cap;
  L.dsq = L.phi + PHIC * a.sig_cap;
  L.Mm = L.dsq + a.nu_cap;
  L.Sm = L.Mm + 64;
  L.wit = reinterpret_cast<int*>(L.Sm + 64);
  L.sbase = L.wit + 8;
  L.sgeo = L.sbase + 48;
  L.red = L.Sm + 64 + 40;
  double* uni = L.red + RED * 36;
  L.tt = uni;
  L.pbuf = uni;
  return L;
}

// Stage the S_k values of E's corners on E's closure into LDS (one coalesced
// pass over the closure's CSR rows; corners that are not in a row read 0).
// With skip_own the entity's own cells are left unset (the forward solve
// writes them).
template <int BLOCK>
__device__ void load_phi_table(const EntDesc& E, const LocalParams& a, double* phi, bool skip_own,
                               const double* vals = nullptr) {
  const double* pv = vals ? vals : a.pval;
  const int ncl = E.cext[0] * E.cext[1] * E.cext[2];
  const int nc = E.nc;
  for (int i = threadIdx.x; i < ncl; i += BLOCK) {
    const int lx = i % E.cext[0];
    const int t = i / E.cext[0];
    const int ly = t % E.cext[1];
    const int lz = t / E.cext[1];
    const int ox = E.clo[0] + lx - E.ulo[0], oy = E.clo[1] + ly - E.ulo[1], oz = E.clo[2] + lz - E.ulo[2];
    const bool own = ox >= 0 && ox < E.uext[0] && oy >= 0 && oy < E.uext[1] && oz >= 0 && oz < E.uext[2];
    if (skip_own && own) continue;
    const int gid = (E.clo[0] + lx) + a.g.s1 * (E.clo[1] + ly) + a.g.s2 * (E.clo[2] + lz);
    const int r0 = a.prow[gid], r1 = a.prow[gid + 1];
    double v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = 0.0;
    if (own) {
      // an own cell's row holds exactly the entity's corners, in corner
      // order: no column matching, all loads at once
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (q < nc) v[q] = pv[r0 + q];
    } else {
      // a closure cell off the own box lies on a lower-dimensional entity:
      // its row holds at most four corners (a face cell), read at once; any
      // further entries in a loop
      int col[4];
      double val[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const bool in = r0 + t < r1;
        col[t] = in ? a.pcol[r0 + t] : -1;
        val[t] = in ? pv[r0 + t] : 0.0;
      }
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (q < nc && E.vid[q] == col[t]) v[q] = val[t];
      for (int e = r0 + 4; e < r1; ++e) {
        const int vid = a.pcol[e];
        const double vv = pv[e];
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (q < nc && E.vid[q] == vid) v[q] = vv;
      }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (q < nc) phi[q * ncl + i] = v[q];
  }
}

// receiver-local own index of the neighbour across direction dd of cell (gcx, gcy, gcz)
__device__ __forceinline__ int receiver_index(const EntDesc& R, int gx, int gy, int gz) {
  return (gx - R.ulo[0]) + R.uext[0] * ((gy - R.ulo[1]) + R.uext[1] * (gz - R.ulo[2]));
}

__device__ __forceinline__ int corner_in(const EntDesc& R, int vid) {
  int ct = -1;
  for (int q = 0; q < R.nc; ++q)
    if (R.vid[q] == vid) ct = q;
  return ct;
}

// ---------------------------------------------------------------------------
// Forward local solves of one entity per workgroup.  Wave w solves corners
// w, w + NWAVE, ... (NCMAX corners at most); each solution goes to S_k and
// into the own-cell entries of the LDS basis table, from which the energy
// block is formed at the end.  Four waves per block (two corners each) keep
// two blocks resident per compute unit, so one block's setup and gathers
// overlap the other's iterations.
template <int NWAVE, int NCMAX, int LMAX>
__device__ __forceinline__ void wave_fwd_body(const LocalParams& a, const EntDesc& E, int eid, double* lds) {
  constexpr int BLOCK = NWAVE * 64;
  const WaveLds S = carve<NWAVE, NCMAX, NWAVE>(a, lds);
  const int nc = E.nc;
  const WGeo w = wave_geo(E, a.g);
  const int ncl = E.cext[0] * E.cext[1] * E.cext[2];
  load_phi_table<BLOCK>(E, a, S.phi, !a.prescribe);
  shared_setup<BLOCK>(E, a.g, a.sig, S.sig, S.dsq, S.tt, w);
  __syncthreads();
  const int wid = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  const int ia0 = lane % w.lw, ib0 = lane / w.lw;
  const bool valid = ia0 < w.Ua && ib0 < w.Ub;
  // the offsets of the S_k rows of the lane's own cells, read ahead of the
  // solves: a store after a solve then waits on no load (a load issued
  // after the previous corner's stores would wait for them too, the vector
  // memory counter being in order)
  int own_row[LMAX];
#pragma unroll
  for (int k = 0; k < LMAX; ++k)
    own_row[k] = (valid && k < w.L) ? a.prow[w.g0 + ia0 * w.ga + ib0 * w.gb + k * w.gc] : 0;
  Column<LMAX> C;
  if (wid < nc && !a.prescribe) load_column<LMAX>(E, w, valid, ia0, ib0, S.tt, C);
  __syncthreads();  // tt is dead from here on; pbuf aliases it
  // scaled right-hand side of corner c: sum over Dirichlet neighbours T phi_c(n)
  auto rhs = [&](int c, int ia, int ib, double (&y)[LMAX]) {
#pragma unroll
    for (int k = 0; k < LMAX; ++k) {
      y[k] = 0.0;
      if (!valid || k >= w.L) continue;
      int fm, um;
      cell_masks(E, w, ia, ib, k, &fm, &um);
      const int ci = w.s0 + ia * w.sa + ib * w.sb + k * w.sc;
      double b = 0.0;
#pragma unroll
      for (int dd = 0; dd < 6; ++dd) {
        if (!((fm >> dd) & 1) || ((um >> dd) & 1)) continue;
        const int sgn = (dd & 1) ? 1 : -1;
        const int cn = ci + sgn * cstr(E, dd >> 1);
        b += harm(S.sig[ci], S.sig[cn]) * S.phi[c * ncl + cn];
      }
      y[k] = b / S.dsq[ia * w.ua + ib * w.ub + k * w.uc];
    }
  };
  // Start vector of a dual block bounded by vertex planes on all three axes:
  // the transfinite (Gordon-Hall) interpolation of corner c's values on the
  // closure boundary, i.e. the sum of the three one-axis linear blends between
  // opposite faces, minus the three two-axis blends between edges, plus the
  // trilinear blend of the eight vertex cells (index coordinates, planes at 0
  // and U+1 on each axis); scaled like the unknowns.  On the 128^3 field it
  // leaves about 4e-4 of the right-hand side as initial residual, against
  // 0.12 for the trilinear Lagrange values.
  const bool guess = E.bounded_mask == 7 && w.L <= LMAX;
  auto coons = [&](int c, int ia, int ib, double (&x0)[LMAX]) {
    const int A = w.Ua + 1, B = w.Ub + 1, Cc = w.L + 1;
    const double* f = S.phi + c * ncl;
    // closure index of closure coordinates (pa, pb, pc); own cell (0,0,0) is (1,1,1)
    auto at = [&](int pa, int pb, int pc) {
      return f[w.s0 + (pa - 1) * w.sa + (pb - 1) * w.sb + (pc - 1) * w.sc];
    };
    const int ja = ia + 1, jb = ib + 1;
    const double xa = double(ja) / A, xb = double(jb) / B;
    // the parts that do not depend on the column position
    const double fc0 = at(ja, jb, 0), fc1 = at(ja, jb, Cc);
    const double e00 = at(ja, 0, 0), e10 = at(ja, B, 0), e01 = at(ja, 0, Cc), e11 = at(ja, B, Cc);
    const double g00 = at(0, jb, 0), g10 = at(A, jb, 0), g01 = at(0, jb, Cc), g11 = at(A, jb, Cc);
    double v[2][2][2];
#pragma unroll
    for (int sa = 0; sa < 2; ++sa)
#pragma unroll
      for (int sb = 0; sb < 2; ++sb)
#pragma unroll
        for (int sc = 0; sc < 2; ++sc) v[sa][sb][sc] = at(sa * A, sb * B, sc * Cc);
#pragma unroll
    for (int k = 0; k < LMAX; ++k) {
      x0[k] = 0.0;
      if (!valid || k >= w.L) continue;
      const int jc = k + 1;
      const double xc = double(jc) / Cc;
      const double pa = (1 - xa) * at(0, jb, jc) + xa * at(A, jb, jc);
      const double pb = (1 - xb) * at(ja, 0, jc) + xb * at(ja, B, jc);
      const double pc = (1 - xc) * fc0 + xc * fc1;
      const double pab = (1 - xa) * ((1 - xb) * at(0, 0, jc) + xb * at(0, B, jc)) +
                         xa * ((1 - xb) * at(A, 0, jc) + xb * at(A, B, jc));
      const double pbc = (1 - xb) * ((1 - xc) * e00 + xc * e01) + xb * ((1 - xc) * e10 + xc * e11);
      const double pac = (1 - xa) * ((1 - xc) * g00 + xc * g01) + xa * ((1 - xc) * g10 + xc * g11);
      const double pabc =
          (1 - xa) * ((1 - xb) * ((1 - xc) * v[0][0][0] + xc * v[0][0][1]) +
                      xb * ((1 - xc) * v[0][1][0] + xc * v[0][1][1])) +
          xa * ((1 - xb) * ((1 - xc) * v[1][0][0] + xc * v[1][0][1]) + xb * ((1 - xc) * v[1][1][0] + xc * v[1][1][1]));
      const double xv = pa + pb + pc - pab - pbc - pac + pabc;
      x0[k] = xv * S.dsq[ia * w.ua + ib * w.ub + k * w.uc];
    }
  };
  // The same for an entity of one cell a lane (faces, and dual blocks of a
  // 2-D grid) bounded on both of its open axes: the bilinear (Coons) blend
  // of the corner's values on the four sides of the closure.
  const bool guess2 = LMAX == 1 && w.L == 1 && E.bounded_mask == E.open_mask && __popc(E.open_mask) == 2;
  auto coons2 = [&](int c, int ia, int ib, double (&x0)[LMAX]) {
#pragma unroll
    for (int k = 0; k < LMAX; ++k) x0[k] = 0.0;
    if (c >= nc || !valid) return;
    const int A = w.Ua + 1, B = w.Ub + 1;
    const double* f = S.phi + c * ncl;
    auto at = [&](int pa, int pb) { return f[w.s0 + (pa - 1) * w.sa + (pb - 1) * w.sb]; };
    const int ja = ia + 1, jb = ib + 1;
    const double xa = double(ja) / A, xb = double(jb) / B;
    const double pa = (1 - xa) * at(0, jb) + xa * at(A, jb);
    const double pb = (1 - xb) * at(ja, 0) + xb * at(ja, B);
    const double pab = (1 - xa) * ((1 - xb) * at(0, 0) + xb * at(0, B)) + xa * ((1 - xb) * at(A, 0) + xb * at(A, B));
    x0[0] = (pa + pb - pab) * S.dsq[ia * w.ua + ib * w.ub];
  };
  // corner c's values on the own cells (unscaled solution, or the Lagrange
  // values of a prescribed entity) to S_k and to the LDS basis table
  auto store = [&](int c, int ia, int ib, const double (&y)[LMAX]) {
#pragma unroll
    for (int k = 0; k < LMAX; ++k) {
      if (!valid || k >= w.L) continue;
      const int u = ia * w.ua + ib * w.ub + k * w.uc;
      const int gid = w.g0 + ia * w.ga + ib * w.gb + k * w.gc;
      const int ci = w.s0 + ia * w.sa + ib * w.sb + k * w.sc;
      double x;
      if (a.prescribe) {
        int gcv[3];
        gcv[0] = gid % a.g.n[0];
        gcv[1] = (gid / a.g.n[0]) % a.g.n[1];
        gcv[2] = gid / (a.g.n[0] * a.g.n[1]);
        x = lagrange_value(E, gcv, c);
      } else {
        x = y[k] / S.dsq[u];
      }
      a.pval[own_row[k] + c] = x;
      S.phi[c * ncl + ci] = x;
    }
  };
  if constexpr (NWAVE == 1) {
    // all (at most four) corners in lockstep in the one wave
    static_assert(NCMAX == 4, "one wave per entity takes four corners");
    double y[4][LMAX];
    if (!a.prescribe) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if (c < nc) {
          rhs(c, ia0, ib0, y[c]);
        } else {
#pragma unroll
          for (int k = 0; k < LMAX; ++k) y[c][k] = 0.0;
        }
      }
      int its[4];
      bool ok[4];
      double res2 = 0.0;
      if (guess2) {
        double x0[4][LMAX];
#pragma unroll
        for (int c = 0; c < 4; ++c) coons2(c, ia0, ib0, x0[c]);
        wave_cg4<LMAX>(w, valid, ia0, ib0, C, y, S.pbuf, a.plane_cap, a.rtol * a.rtol, a.maxit, its, ok, &x0,
                       &res2);
      } else {
        wave_cg4<LMAX>(w, valid, ia0, ib0, C, y, S.pbuf, a.plane_cap, a.rtol * a.rtol, a.maxit, its, ok, nullptr,
                       &res2);
      }
      if (lane == 0) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          if (c >= nc) continue;
          S.wit[c] = its[c];
          if (!ok[c]) atomicAdd(a.status + kStLocalNoconv, 1);
        }
        if (a.ent_res) a.ent_res[size_t(eid) * 8] = res2;
      }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (c < nc) store(c, ia0, ib0, y[c]);
  } else {
    double* pbuf = S.pbuf + wid * a.plane_cap;
#pragma unroll 1
    for (int c = wid; c < nc; c += NWAVE) {
      // opaque copies of the lane coordinates: what derives from them is
      // recomputed in each pass instead of being kept live across passes
      int ia = ia0, ib = ib0;
      asm volatile("" : "+v"(ia), "+v"(ib));
      double y[LMAX];
      if (!a.prescribe) {
        rhs(c, ia, ib, y);
        bool ok = true;
        int it;
        double res2 = 0.0;
        if (guess) {
          double x0[LMAX];
          coons(c, ia, ib, x0);
          it = wave_cg<LMAX>(w, valid, ia, ib, C, y, pbuf, a.rtol * a.rtol, a.maxit, &ok, &x0, &res2);
        } else {
          it = wave_cg<LMAX>(w, valid, ia, ib, C, y, pbuf, a.rtol * a.rtol, a.maxit, &ok, nullptr, &res2);
        }
        if (lane == 0) {
          S.wit[c] = it;
          if (!ok) atomicAdd(a.status + kStLocalNoconv, 1);
          if (a.ent_res) a.ent_res[size_t(eid) * 8 + c] = res2;
        }
        wave_sync_lds();
      }
      store(c, ia, ib, y);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0 && a.ent_it) {
    int itm = 0;
    unsigned long long wk = 0;
    if (!a.prescribe)
      for (int q = 0; q < nc; ++q) {
        itm = max(itm, S.wit[q]);
        wk += (unsigned long long)S.wit[q] * E.nu;
      }
    a.ent_it[eid] = itm;
    if (a.ent_work) a.ent_work[eid] += wk;
  }
  // energy block K_E = sum over the touched fluxes T dphi dphi^T: one thread
  // per own cell and its owned fluxes, then a fixed-order block reduction
  constexpr int NQ = NCMAX * (NCMAX + 1) / 2;
  double kacc[NQ];
#pragma unroll
  for (int i = 0; i < NQ; ++i) kacc[i] = 0.0;
  const int nflux = owned_flux_count(E);
  for (int item = threadIdx.x; item < nflux; item += BLOCK) {
    const OwnedFlux f = owned_flux(E, a.g, w.g0, item);
    if (!f.valid) continue;
    const int ci = f.ci, cn = f.ci + f.sgn * cstr(E, f.ax);
    const double T = harm(S.sig[ci], S.sig[cn]);
    double dp[NCMAX];
#pragma unroll
    for (int q = 0; q < NCMAX; ++q) dp[q] = q < nc ? S.phi[q * ncl + ci] - S.phi[q * ncl + cn] : 0.0;
    int qq = 0;
#pragma unroll
    for (int q = 0; q < NCMAX; ++q) {
      const double tq = T * dp[q];
#pragma unroll
      for (int q2 = q; q2 < NCMAX; ++q2) kacc[qq++] += tq * dp[q2];
    }
  }
  block_sum<NWAVE, NQ>(kacc, S.red);
  // K_E[q][q2] from the upper triangle, row q at offset q*NCMAX - q(q-1)/2
  if (threadIdx.x < nc * nc) {
    const int q = threadIdx.x / nc, q2 = threadIdx.x % nc;
    const int lo = min(q, q2), hi = max(q, q2);
    a.kent[E.kbase + threadIdx.x] = S.red[lo * NCMAX - lo * (lo - 1) / 2 + (hi - lo)];
  }
}

// A dual block of U^3 own cells bounded by vertex planes on every axis (the
// full blocks of coarsening U + 1): the geometry fields every helper reads
// become compile-time constants, so index arithmetic, plane offsets and
// neighbour masks fold away; position, corners and table offsets stay the
// entity's.
template <int U>
__device__ __forceinline__ EntDesc full_block(const EntDesc& src) {
  EntDesc E = src;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    E.uext[k] = U;
    E.cext[k] = U + 2;
    E.clo[k] = src.ulo[k] - 1;
  }
  E.open_mask = 7;
  E.bounded_mask = 7;
  E.nc = 8;
  E.nu = U * U * U;
  return E;
}

// A face of U x U own cells on a plane of axis NAX, bounded by vertex
// planes on both of its open axes (the full faces of coarsening U + 1; on a
// 2-D grid, NAX = 2, the full dual blocks): compile-time geometry as for the
// full blocks.
template <int U, int NAX>
__device__ __forceinline__ EntDesc full_face(const EntDesc& src) {
  EntDesc E = src;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    E.uext[k] = k == NAX ? 1 : U;
    E.cext[k] = k == NAX ? 1 : U + 2;
    E.clo[k] = k == NAX ? src.ulo[k] : src.ulo[k] - 1;
  }
  E.open_mask = 7 & ~(1 << NAX);
  E.bounded_mask = 7 & ~(1 << NAX);
  E.nc = 4;
  E.nu = U * U;
  return E;
}

// Plane axis of E if E has the shape full_face<U, axis> fixes, else -1
// (the host orders the face list by the same test).
template <int U>
__device__ __forceinline__ int full_face_axis(const EntDesc& E) {
  if (E.nc != 4 || E.nu != U * U || E.bounded_mask != E.open_mask) return -1;
  int nax = -1;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if ((E.open_mask >> k) & 1) {
      if (E.uext[k] != U || E.cext[k] != U + 2 || E.clo[k] != E.ulo[k] - 1) return -1;
    } else {
      if (nax >= 0 || E.uext[k] != 1 || E.cext[k] != 1 || E.clo[k] != E.ulo[k]) return -1;
      nax = k;
    }
  }
  return nax;
}

// Whether E has the shape full_block<U> fixes (the host lists the full
// blocks by the same test).
template <int U>
__device__ __forceinline__ bool is_full_block(const EntDesc& E) {
  if (E.open_mask != 7 || E.bounded_mask != 7 || E.nc != 8 || E.nu != U * U * U) return false;
#pragma unroll
  for (int k = 0; k < 3; ++k)
    if (E.uext[k] != U || E.cext[k] != U + 2 || E.clo[k] != E.ulo[k] - 1) return false;
  return true;
}

// FULLU codes of the kernels: 0 any entity, U full U^3 blocks only,
// faces_code(U) any face, the full U x U faces through a body of their own
// for each plane axis (one launch for all: a face's wave lives for tens of
// microseconds, so a launch per axis would leave the device part-empty in
// every launch's tail); blocks_code(U) any dual block, the full U^3 ones
// through their own body (one launch for the full and the other blocks, for
// the same reason).
constexpr int faces_code(int u) { return 64 + u; }
constexpr int blocks_code(int u) { return 128 + u; }

// Run BODY on eid's entity with the geometry the launch fixes.
template <int FULLU, typename Body>
__device__ __forceinline__ void with_shape(const LocalParams& a, int eid, Body&& body) {
  const EntDesc& G = a.ents[eid];
  if constexpr (FULLU >= 128) {
    constexpr int U = FULLU - 128;
    if (__builtin_amdgcn_readfirstlane(is_full_block<U>(G) ? 1 : 0))
      body(full_block<U>(G));
    else
      body(G);
  } else if constexpr (FULLU >= 64) {
    constexpr int U = FULLU - 64;
    const int nax = __builtin_amdgcn_readfirstlane(full_face_axis<U>(G));
    if (nax == 0)
      body(full_face<U, 0>(G));
    else if (nax == 1)
      body(full_face<U, 1>(G));
    else if (nax == 2)
      body(full_face<U, 2>(G));
    else
      body(G);
  } else if constexpr (FULLU > 0) {
    body(full_block<FULLU>(G));
  } else {
    body(G);
  }
}

template <int NWAVE, int NCMAX, int LMAX, int FULLU>
__device__ __forceinline__ void wave_fwd_one(const LocalParams& a, int eid, double* lds) {
  with_shape<FULLU>(a, eid, [&](const EntDesc& E) { wave_fwd_body<NWAVE, NCMAX, LMAX>(a, E, eid, lds); });
}

// FULLU = 0: any entity of the launch; FULLU = U: only full U^3 blocks;
// FULLU = faces_code(U): faces, the full U x U ones with their shape fixed.
// MULTI: a fixed grid strides over (problem, entity) items of many problems.
// The one-wave (face) launches ask for five waves a SIMD, i.e. at most 96
// VGPRs: the few registers that then spill cost less than the fifth wave
// gains in hiding the latency of the face's memory reads.
template <int NWAVE, int NCMAX, int LMAX, int FULLU = 0, bool MULTI = false>
__global__ __launch_bounds__(NWAVE * 64, (NWAVE == 1 && !MULTI ? 5 : (NWAVE <= 4 ? 2 : 1))) void k_wave_fwd(LocalParams a) {
  extern __shared__ double lds[];
  if constexpr (MULTI) {
    for (int it = blockIdx.x; it < a.nent; it += gridDim.x) {
      const int2 w = a.items[it];
      wave_fwd_one<NWAVE, NCMAX, LMAX, FULLU>(a.multi[w.x], w.y, lds);
      __syncthreads();  // the next item reuses the LDS tables
    }
  } else {
    wave_fwd_one<NWAVE, NCMAX, LMAX, FULLU>(a, ent_index(a), lds);
  }
}

// ---------------------------------------------------------------------------
// Adjoint local solves (source-reduced, transposed) of one entity per
// workgroup, corners distributed over the waves as in the forward kernel.
// y_c = sum_q (M + M^T)_{qc} phi_q is formed where it is needed from the LDS
// basis table; each corner's adjoint solution mu_c goes to the entity's
// slice of a global scratch (it stays in L2) for the flux weights.
template <int NWAVE, int NCMAX, int LMAX>
__device__ __forceinline__ void wave_adj_body(const LocalParams& a, const EntDesc& E, int eid, double* lds) {
  constexpr int BLOCK = NWAVE * 64;
  const WaveLds S = carve<NWAVE, NCMAX, NWAVE>(a, lds);
  const int nc = E.nc;
  const long long N = (long long)a.g.n[0] * a.g.n[1] * a.g.n[2];
  const WGeo w = wave_geo(E, a.g);
  const int ncl = E.cext[0] * E.cext[1] * E.cext[2];
  // the arrays of the descriptor that are indexed per lane are read from
  // memory: indexed so, a register copy of the descriptor (the shapes fixed
  // at compile time) would live in scratch memory
  const EntDesc& D = a.ents[eid];
  // mu_c on own cells: for a one-wave entity in its plane buffers, dead once
  // the lockstep solves of its corners are done (4 nu <= 6 nu of that
  // region); else in the entity's slice of a global scratch
  double* mus = NWAVE == 1 ? S.pbuf : a.mu_scratch + size_t(eid) * NCMAX * a.nu_cap;
  load_phi_table<BLOCK>(E, a, S.phi, false);
  // M_E = sum_j t_j lambda_j^T on the corners; t and lambda of the corners
  // are staged, a chunk of sources at a time, through the plane buffers
  // before the transmissibilities take that space
  {
    double* tl = S.pbuf;
    const int cap = max(1, a.uni_cap / (2 * nc));  // sources a chunk
    double s = 0.0;
    for (int j0 = 0; j0 < a.ns; j0 += cap) {
      const int nj = min(cap, a.ns - j0);
      for (int i = threadIdx.x; i < 2 * nc * nj; i += BLOCK) {
        const int which = i / (nc * nj), r = i % (nc * nj), q = r / nj, j = r % nj;
        const double* src = which ? a.lam : a.t;
        tl[i] = src[size_t(j0 + j) * a.ncoarse + D.vid[q]];
      }
      __syncthreads();
      if (threadIdx.x < nc * nc) {
        const int q = threadIdx.x / nc, q2 = threadIdx.x % nc;
        for (int j = 0; j < nj; ++j) s += tl[q * nj + j] * tl[(nc + q2) * nj + j];
      }
      __syncthreads();
    }
    if (threadIdx.x < nc * nc) S.Mm[threadIdx.x] = s;
  }
  // an entity with no electrode loads and no pushes from above has zero
  // adjoint loads (dual blocks off the electrodes): no local operator, no
  // solve, only the pushes of y_c and the flux weights
  const bool loaded = a.solve_adj && (E.nslot > 0 || E.eptr1 > E.eptr0);
  shared_setup<BLOCK>(E, a.g, a.sig, S.sig, S.dsq, S.tt, w, loaded);
  __syncthreads();
  if (threadIdx.x < nc * nc) {
    const int q = threadIdx.x / nc, q2 = threadIdx.x % nc;
    S.Sm[threadIdx.x] = S.Mm[q * nc + q2] + S.Mm[q2 * nc + q];
  }
  // receiver slots of the pushes across each side of the closure
  if (threadIdx.x < 48) {
    const int side = threadIdx.x >> 3, c = threadIdx.x & 7;
    const int te = D.side_ent[side];
    int base = -1;
    if (a.push && te >= 0 && c < nc) {
      const EntDesc& R = a.recv[te];
      const int ct = corner_in(R, D.vid[c]);
      if (ct >= 0) base = R.inbase + (D.side_slot[side] * R.nc + ct) * R.nu;
      if (c == 0) {
        const int s1 = R.uext[0], s2 = R.uext[0] * R.uext[1];
        S.sgeo[3 * side + 0] = s1;
        S.sgeo[3 * side + 1] = s2;
        S.sgeo[3 * side + 2] = -(R.ulo[0] + s1 * R.ulo[1] + s2 * R.ulo[2]);
      }
    }
    S.sbase[threadIdx.x] = base;
  }
  const int wid = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  const int ia0 = lane % w.lw, ib0 = lane / w.lw;
  const bool valid = ia0 < w.Ua && ib0 < w.Ub;
  const bool any = wid < nc && loaded;
  __syncthreads();
  Column<LMAX> C;
  if (any) load_column<LMAX>(E, w, valid, ia0, ib0, S.tt, C);
  __syncthreads();  // tt is dead; pbuf aliases it
  // load z_c on own cells: the pushes of the entities above and the
  // electrode loads, scaled.  The -(A^E y_c) part of the load vanishes on
  // own cells: y_c = sum_q (M + M^T)_{qc} phi_q combines the corner bases,
  // and each of them satisfies the entity's local problem there (to the
  // local solve tolerance).  Across the fluxes to Dirichlet neighbours y_c
  // enters the pushes, whose y-part is written here.
  auto load = [&](int c, int ia, int ib, double (&y)[LMAX]) {
    // y_c at closure cell ci (column c of M + M^T read from LDS)
    auto ycl = [&](int ci) {
      double v = 0.0;
#pragma unroll
      for (int q = 0; q < NCMAX; ++q)
        if (q < nc) v += S.Sm[q * nc + c] * S.phi[q * ncl + ci];
      return v;
    };
#pragma unroll
    for (int k = 0; k < LMAX; ++k) {
      y[k] = 0.0;
      if (!valid || k >= w.L) continue;
      int fm, um;
      cell_masks(E, w, ia, ib, k, &fm, &um);
      const int ci = w.s0 + ia * w.sa + ib * w.sb + k * w.sc;
      const int u = ia * w.ua + ib * w.ub + k * w.uc;
      double z = 0.0;
      for (int s = 0; s < E.nslot; ++s) z += a.inbuf[E.inbase + (s * nc + c) * E.nu + u];
      for (int e = E.eptr0; e < E.eptr1; ++e)
        if (a.eloc[e] == u) z += a.sload[a.eidx[e] * 8 + c];
      if (fm & ~um & 63) {
        const double yu = ycl(ci);
#pragma unroll
        for (int dd = 0; dd < 6; ++dd) {
          if (!((fm >> dd) & 1) || ((um >> dd) & 1)) continue;
          const int base = S.sbase[dd * 8 + c];
          if (base < 0) continue;
          const int sgn = (dd & 1) ? 1 : -1;
          const int cn = ci + sgn * cstr(E, dd >> 1);
          const double T = harm(S.sig[ci], S.sig[cn]);
          int gc3[3];
          own_coords(E, w, ia, ib, k, gc3);
          gc3[dd >> 1] += sgn;
          a.outbuf[base + gc3[0] + S.sgeo[3 * dd] * gc3[1] + S.sgeo[3 * dd + 1] * gc3[2] + S.sgeo[3 * dd + 2]] =
              T * (yu - ycl(cn));
        }
      }
      y[k] = loaded ? z / S.dsq[u] : 0.0;
    }
  };
  // mu_c to the scratch; mu-part of the pushes.  A zero load (no
  // electrodes, no pushes from above) gives mu_c = 0 without iterations:
  // nothing to store or push, and the flux weights skip the corner.
  auto finish = [&](int c, int ia, int ib, const double (&y)[LMAX], int it) {
#pragma unroll
    for (int k = 0; k < LMAX; ++k) {
      if (it == 0 || !valid || k >= w.L) continue;
      const int u = ia * w.ua + ib * w.ub + k * w.uc;
      const double mu = y[k] / S.dsq[u];
      mus[c * a.nu_cap + u] = mu;
      if (!a.push) continue;
      int fm, um;
      cell_masks(E, w, ia, ib, k, &fm, &um);
      const int ci = w.s0 + ia * w.sa + ib * w.sb + k * w.sc;
#pragma unroll
      for (int dd = 0; dd < 6; ++dd) {
        if (!((fm >> dd) & 1) || ((um >> dd) & 1)) continue;
        const int base = S.sbase[dd * 8 + c];
        if (base < 0) continue;
        const int sgn = (dd & 1) ? 1 : -1;
        const double T = harm(S.sig[ci], S.sig[ci + sgn * cstr(E, dd >> 1)]);
        int gc3[3];
        own_coords(E, w, ia, ib, k, gc3);
        gc3[dd >> 1] += sgn;
        // the same thread stored the y-part of this slot before the solve:
        // a no-return atomic add finishes the sum without a load round trip
        unsafeAtomicAdd(a.outbuf + base + gc3[0] + S.sgeo[3 * dd] * gc3[1] + S.sgeo[3 * dd + 1] * gc3[2] +
                            S.sgeo[3 * dd + 2],
                        T * mu);
      }
    }
  };
  if constexpr (NWAVE == 1) {
    // all (at most four) corners in lockstep in the one wave
    static_assert(NCMAX == 4, "one wave per entity takes four corners");
    if (a.solve_adj) {
      double y[4][LMAX];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if (c < nc) {
          load(c, ia0, ib0, y[c]);
        } else {
#pragma unroll
          for (int k = 0; k < LMAX; ++k) y[c][k] = 0.0;
        }
      }
      __threadfence_block();  // the y-part stores complete before the mu-part adds below
      int its[4] = {0, 0, 0, 0};
      bool ok[4] = {true, true, true, true};
      double res2 = 0.0;
      if (loaded)
        wave_cg4<LMAX>(w, valid, ia0, ib0, C, y, S.pbuf, a.plane_cap, a.rtol * a.rtol, a.maxit, its, ok, nullptr,
                       &res2);
      if (lane == 0) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          if (c >= nc) continue;
          S.wit[c] = its[c];
          if (!ok[c]) atomicAdd(a.status + kStLocalNoconv, 1);
        }
        if (a.ent_res) a.ent_res[size_t(eid) * 8] = res2;
      }
#pragma unroll
      for (int c = 0; c < 4; ++c)
        if (c < nc) finish(c, ia0, ib0, y[c], its[c]);
    }
  } else {
    double* pbuf = S.pbuf + wid * a.plane_cap;
  #pragma unroll 1
    for (int c = a.solve_adj ? wid : nc; c < nc; c += NWAVE) {
      // opaque copies of the lane coordinates (see the forward kernel)
      int ia = ia0, ib = ib0;
      asm volatile("" : "+v"(ia), "+v"(ib));
      double sc[NCMAX];  // column c of M + M^T
  #pragma unroll
      for (int q = 0; q < NCMAX; ++q) sc[q] = q < nc ? S.Sm[q * nc + c] : 0.0;
      auto ycl = [&](int ci) {
        double v = 0.0;
  #pragma unroll
        for (int q = 0; q < NCMAX; ++q)
          if (q < nc) v += sc[q] * S.phi[q * ncl + ci];
        return v;
      };
      double y[LMAX];
      // load z_c on own cells: the pushes of the entities above and the
      // electrode loads, scaled.  The -(A^E y_c) part of the load vanishes on
      // own cells: y_c combines the corner bases, and each of them satisfies
      // the entity's local problem there (to the local solve tolerance).
      // Across the fluxes to Dirichlet neighbours y_c enters the pushes, whose
      // y-part is written here.
  #pragma unroll
      for (int k = 0; k < LMAX; ++k) {
        y[k] = 0.0;
        if (!valid || k >= w.L) continue;
        int fm, um;
        cell_masks(E, w, ia, ib, k, &fm, &um);
        const int ci = w.s0 + ia * w.sa + ib * w.sb + k * w.sc;
        const int u = ia * w.ua + ib * w.ub + k * w.uc;
        double z = 0.0;
        for (int s = 0; s < E.nslot; ++s) z += a.inbuf[E.inbase + (s * nc + c) * E.nu + u];
        for (int e = E.eptr0; e < E.eptr1; ++e)
          if (a.eloc[e] == u) z += a.sload[a.eidx[e] * 8 + c];
        if (fm & ~um & 63) {
          const double yu = ycl(ci);
  #pragma unroll
          for (int dd = 0; dd < 6; ++dd) {
            if (!((fm >> dd) & 1) || ((um >> dd) & 1)) continue;
            const int base = S.sbase[dd * 8 + c];
            if (base < 0) continue;
            const int sgn = (dd & 1) ? 1 : -1;
            const int cn = ci + sgn * cstr(E, dd >> 1);
            const double T = harm(S.sig[ci], S.sig[cn]);
            int gc3[3];
            own_coords(E, w, ia, ib, k, gc3);
            gc3[dd >> 1] += sgn;
            a.outbuf[base + gc3[0] + S.sgeo[3 * dd] * gc3[1] + S.sgeo[3 * dd + 1] * gc3[2] + S.sgeo[3 * dd + 2]] =
                T * (yu - ycl(cn));
          }
        }
        y[k] = loaded ? z / S.dsq[u] : 0.0;
      }
      __threadfence_block();  // the y-part stores complete before the mu-part adds below
      bool ok = true;
      double res2 = 0.0;
      const int it =
          loaded ? wave_cg<LMAX>(w, valid, ia, ib, C, y, pbuf, a.rtol * a.rtol, a.maxit, &ok, nullptr, &res2) : 0;
      if (lane == 0) {
        S.wit[c] = it;
        if (!ok) atomicAdd(a.status + kStLocalNoconv, 1);
        if (a.ent_res) a.ent_res[size_t(eid) * 8 + c] = res2;
      }
      // mu_c to the scratch; mu-part of the pushes.  A zero load (no
      // electrodes, no pushes from above) gives mu_c = 0 without iterations:
      // nothing to store or push, and the flux weights skip the corner.
  #pragma unroll
      for (int k = 0; k < LMAX; ++k) {
        if (it == 0 || !valid || k >= w.L) continue;
        const int u = ia * w.ua + ib * w.ub + k * w.uc;
        const double mu = y[k] / S.dsq[u];
        mus[c * a.nu_cap + u] = mu;
        if (!a.push) continue;
        int fm, um;
        cell_masks(E, w, ia, ib, k, &fm, &um);
        const int ci = w.s0 + ia * w.sa + ib * w.sb + k * w.sc;
  #pragma unroll
        for (int dd = 0; dd < 6; ++dd) {
          if (!((fm >> dd) & 1) || ((um >> dd) & 1)) continue;
          const int base = S.sbase[dd * 8 + c];
          if (base < 0) continue;
          const int sgn = (dd & 1) ? 1 : -1;
          const double T = harm(S.sig[ci], S.sig[ci + sgn * cstr(E, dd >> 1)]);
          int gc3[3];
          own_coords(E, w, ia, ib, k, gc3);
          gc3[dd >> 1] += sgn;
          // the same thread stored the y-part of this slot before the solve:
          // a no-return atomic add finishes the sum without a load round trip
          unsafeAtomicAdd(a.outbuf + base + gc3[0] + S.sgeo[3 * dd] * gc3[1] + S.sgeo[3 * dd + 1] * gc3[2] +
                              S.sgeo[3 * dd + 2],
                          T * mu);
        }
      }
      wave_sync_lds();  // the next corner's CG rewrites this wave's buffer
    }
  }
  if constexpr (NWAVE > 1) __threadfence_block();  // mu_c in global memory, read by the other waves
  __syncthreads();
  if (threadIdx.x == 0 && a.ent_it) {
    int itm = 0;
    unsigned long long wk = 0;
    if (a.solve_adj)
      for (int q = 0; q < nc; ++q) {
        itm = max(itm, S.wit[q]);
        wk += (unsigned long long)S.wit[q] * E.nu;
      }
    a.ent_it[eid] = itm;
    if (a.ent_work) a.ent_work[eid] += wk;
  }
  // flux weights W_f = -dphi^T M dphi - sum_c (mu_c(u) - mu_c(n)) dphi_c for
  // owned fluxes; the quadratic form uses the symmetric part of M (upper
  // triangle, off-diagonal entries doubled), held in registers
  constexpr int NQ = NCMAX * (NCMAX + 1) / 2;
  double mh[NQ];
  {
    int qq = 0;
#pragma unroll
    for (int q = 0; q < NCMAX; ++q)
#pragma unroll
      for (int q2 = q; q2 < NCMAX; ++q2) {
        mh[qq] = (q < nc && q2 < nc) ? (q == q2 ? S.Mm[q * nc + q] : S.Sm[q * nc + q2]) : 0.0;
        ++qq;
      }
  }
  const int nflux = owned_flux_count(E);
  for (int item = threadIdx.x; item < nflux; item += BLOCK) {
    const OwnedFlux f = owned_flux(E, a.g, w.g0, item);
    if (!f.valid) continue;
    const int ci = f.ci, u = f.u, gid = f.gid;
    const int cn = ci + f.sgn * cstr(E, f.ax);
    const int un = u + f.sgn * ustr(E, f.ax);
    const int gn = gid + f.sgn * gstr(a.g, f.ax);
    double dp[NCMAX];
#pragma unroll
    for (int q = 0; q < NCMAX; ++q) dp[q] = q < nc ? S.phi[q * ncl + ci] - S.phi[q * ncl + cn] : 0.0;
    double wv = 0.0;
    int qq = 0;
#pragma unroll
    for (int q = 0; q < NCMAX; ++q) {
      double mq = 0.0;
#pragma unroll
      for (int q2 = q; q2 < NCMAX; ++q2) mq += mh[qq++] * dp[q2];
      wv -= dp[q] * mq;
    }
    if (a.solve_adj) {
#pragma unroll
      for (int q = 0; q < NCMAX; ++q) {
        if (q >= nc || S.wit[q] == 0) continue;
        const double mun = f.own ? mus[q * a.nu_cap + un] : 0.0;
        wv -= (mus[q * a.nu_cap + u] - mun) * dp[q];
      }
    }
    a.W[f.ax * N + (f.sgn > 0 ? gid : gn)] = wv;
  }
}


template <int NWAVE, int NCMAX, int LMAX, int FULLU>
__device__ __forceinline__ void wave_adj_one(const LocalParams& a, int eid, double* lds) {
  with_shape<FULLU>(a, eid, [&](const EntDesc& E) { wave_adj_body<NWAVE, NCMAX, LMAX>(a, E, eid, lds); });
}

template <int NWAVE, int NCMAX, int LMAX, int FULLU = 0, bool MULTI = false>
__global__ __launch_bounds__(NWAVE * 64, (NWAVE == 1 && !MULTI ? 5 : (NWAVE <= 4 ? 2 : 1))) void k_wave_adj(LocalParams a) {
  extern __shared__ double lds[];
  if constexpr (MULTI) {
    for (int it = blockIdx.x; it < a.nent; it += gridDim.x) {
      const int2 w = a.items[it];
      wave_adj_one<NWAVE, NCMAX, LMAX, FULLU>(a.multi[w.x], w.y, lds);
      __syncthreads();
    }
  } else {
    wave_adj_one<NWAVE, NCMAX, LMAX, FULLU>(a, ent_index(a), lds);
  }
}

// ---------------------------------------------------------------------------
// Tangent of the face / dual-block basis along dm (Sec. 4.5, forward mode):
// for each corner c, A^E_UU dphi_c = -(dA^E phi_c)_U - A^E_UB dphi_c|_B, with
// dA^E the derivative of the entity's reduced operator along dm and dphi_c|_B
// the tangent of the lower entities (already in dS); then the tangent energy
// block dK_E = sum over the touched fluxes of dT dphi dphi^T +
// T (d(dphi) dphi^T + dphi d(dphi)^T).  Prescribed (Lagrange) entities have
// dphi = 0 and only the dT term.
template <int NWAVE, int NCMAX, int LMAX>
__global__ __launch_bounds__(NWAVE * 64) void k_wave_tan(LocalParams a) {
  extern __shared__ double lds[];
  constexpr int BLOCK = NWAVE * 64;
  const EntDesc& E = a.ents[ent_index(a)];
  const int nc = E.nc;
  const WGeo w = wave_geo(E, a.g);
  const int ncl = E.cext[0] * E.cext[1] * E.cext[2];
  // LDS: sig, phi (8 ncl), dphi (8 ncl), dm (ncl), dsq, small tables, plane buffers
  WaveLds S = carve<NWAVE>(a, lds);
  double* dphi = lds + size_t(9) * a.sig_cap + a.nu_cap + 128 + 40 + 8 * 36 + a.uni_cap;
  double* dmv = dphi + 8 * a.sig_cap;
  load_phi_table<BLOCK>(E, a, S.phi, false);
  load_phi_table<BLOCK>(E, a, dphi, false, a.dpval);
  for (int i = threadIdx.x; i < ncl; i += BLOCK) {
    const int lx = i % E.cext[0], t = i / E.cext[0];
    const int ly = t % E.cext[1], lz = t / E.cext[1];
    dmv[i] = a.dm[(E.clo[0] + lx) + a.g.s1 * (E.clo[1] + ly) + a.g.s2 * (E.clo[2] + lz)];
  }
  shared_setup<BLOCK>(E, a.g, a.sig, S.sig, S.dsq, S.tt, w);
  __syncthreads();
  const int wid = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  const int ia0 = lane % w.lw, ib0 = lane / w.lw;
  const bool valid = ia0 < w.Ua && ib0 < w.Ub;
  Column<LMAX> C;
  if (wid < nc && !a.prescribe) load_column<LMAX>(E, w, valid, ia0, ib0, S.tt, C);
  __syncthreads();  // tt is dead; pbuf aliases it
  double* pbuf = S.pbuf + wid * a.plane_cap;
  auto dT = [&](int ci, int cn) {
    return dharm(S.sig[ci], S.sig[cn]) * dmv[ci] + dharm(S.sig[cn], S.sig[ci]) * dmv[cn];
  };
#pragma unroll 1
  for (int c = wid; c < nc; c += NWAVE) {
    int ia = ia0, ib = ib0;
    asm volatile("" : "+v"(ia), "+v"(ib));
    double y[LMAX];
    if (!a.prescribe) {
#pragma unroll
      for (int k = 0; k < LMAX; ++k) {
        y[k] = 0.0;
        if (!valid || k >= w.L) continue;
        int fm, um;
        cell_masks(E, w, ia, ib, k, &fm, &um);
        const int ci = w.s0 + ia * w.sa + ib * w.sb + k * w.sc;
        const double pc = S.phi[c * ncl + ci];
        double b = 0.0;
#pragma unroll
        for (int dd = 0; dd < 6; ++dd) {
          if (!((fm >> dd) & 1)) continue;
          const int sgn = (dd & 1) ? 1 : -1;
          const int cn = ci + sgn * cstr(E, dd >> 1);
          b -= dT(ci, cn) * (pc - S.phi[c * ncl + cn]);
          if (!((um >> dd) & 1)) b += harm(S.sig[ci], S.sig[cn]) * dphi[c * ncl + cn];
        }
        y[k] = b / S.dsq[ia * w.ua + ib * w.ub + k * w.uc];
      }
      bool ok = true;
      (void)wave_cg<LMAX>(w, valid, ia, ib, C, y, pbuf, a.rtol * a.rtol, a.maxit, &ok);
      if (lane == 0 && !ok) atomicAdd(a.status + kStLocalNoconv, 1);
      wave_sync_lds();
    }
#pragma unroll
    for (int k = 0; k < LMAX; ++k) {
      if (!valid || k >= w.L) continue;
      const int u = ia * w.ua + ib * w.ub + k * w.uc;
      const int gid = w.g0 + ia * w.ga + ib * w.gb + k * w.gc;
      const int ci = w.s0 + ia * w.sa + ib * w.sb + k * w.sc;
      const double x = a.prescribe ? 0.0 : y[k] / S.dsq[u];
      a.dpval[a.prow[gid] + c] = x;
      dphi[c * ncl + ci] = x;
    }
  }
  __syncthreads();
  constexpr int NQ = NCMAX * (NCMAX + 1) / 2;
  double kacc[NQ];
#pragma unroll
  for (int i = 0; i < NQ; ++i) kacc[i] = 0.0;
  const int ncol = w.Ua * w.Ub;
  for (int i = threadIdx.x; i < ncol * w.L; i += BLOCK) {
    const int col = i % ncol, k = i / ncol;
    const int ja = col % w.Ua, jb = col / w.Ua;
    int fm, um;
    cell_masks(E, w, ja, jb, k, &fm, &um);
    const int ci = w.s0 + ja * w.sa + jb * w.sb + k * w.sc;
#pragma unroll
    for (int dd = 0; dd < 6; ++dd) {
      if (!((fm >> dd) & 1)) continue;
      const bool own = (um >> dd) & 1;
      if (!(dd & 1) && own) continue;  // counted from the lower own cell
      const int sgn = (dd & 1) ? 1 : -1;
      const int cn = ci + sgn * cstr(E, dd >> 1);
      const double T = harm(S.sig[ci], S.sig[cn]);
      const double dTf = dT(ci, cn);
      double f[NCMAX], g[NCMAX];
#pragma unroll
      for (int q = 0; q < NCMAX; ++q) {
        f[q] = q < nc ? S.phi[q * ncl + ci] - S.phi[q * ncl + cn] : 0.0;
        g[q] = q < nc ? dphi[q * ncl + ci] - dphi[q * ncl + cn] : 0.0;
      }
      int qq = 0;
#pragma unroll
      for (int q = 0; q < NCMAX; ++q)
#pragma unroll
        for (int q2 = q; q2 < NCMAX; ++q2) kacc[qq++] += dTf * f[q] * f[q2] + T * (g[q] * f[q2] + f[q] * g[q2]);
    }
  }
  block_sum<NWAVE, NQ>(kacc, S.red);
  if (threadIdx.x < nc * nc) {
    const int q = threadIdx.x / nc, q2 = threadIdx.x % nc;
    const int lo = min(q, q2), hi = max(q, q2);
    a.kent[E.kbase + threadIdx.x] = S.red[lo * NCMAX - lo * (lo - 1) / 2 + (hi - lo)];
  }
}

// Galerkin energy blocks from S_k values already in memory and sigma =
// exp(m) of the current model: the frozen basis S_k(m0) of eq. optredfixed, with A_k(m) = S_k^T A(m)
// S_k rebuilt (eq. reducedPDE).  Per entity, K_E = sum over the fine fluxes
// the entity owns of T_f(m) dphi dphi^T over its corners -- the same
// partition of the fluxes and the same sums as the energy phase of the
// local-solve kernels, with phi read from the CSR rows (an own cell's row
// holds the entity's corners in order; a neighbour's row is searched).
template <int NCMAX>
__global__ __launch_bounds__(256) void k_energy_frozen(LocalParams a) {
  constexpr int NQ = NCMAX * (NCMAX + 1) / 2;
  __shared__ double red[4 * NQ];
  const EntDesc& E = a.ents[ent_index(a)];
  const int nc = E.nc;
  const int g0 = E.ulo[0] + a.g.s1 * E.ulo[1] + a.g.s2 * E.ulo[2];
  double kacc[NQ];
#pragma unroll
  for (int i = 0; i < NQ; ++i) kacc[i] = 0.0;
  const int nflux = owned_flux_count(E);
  for (int item = threadIdx.x; item < nflux; item += 256) {
    const OwnedFlux f = owned_flux(E, a.g, g0, item);
    if (!f.valid) continue;
    const int gn = f.gid + f.sgn * gstr(a.g, f.ax);
    const double T = harm(a.sig[f.gid], a.sig[gn]);
    const int r0 = a.prow[f.gid];
    double dp[NCMAX];
#pragma unroll
    for (int q = 0; q < NCMAX; ++q)
      dp[q] = q < nc ? a.pval[r0 + q] - p_lookup(a.prow, a.pcol, a.pval, gn, E.vid[q]) : 0.0;
    int qq = 0;
#pragma unroll
    for (int q = 0; q < NCMAX; ++q) {
      const double tq = T * dp[q];
#pragma unroll
      for (int q2 = q; q2 < NCMAX; ++q2) kacc[qq++] += tq * dp[q2];
    }
  }
  block_sum<4, NQ>(kacc, red);
  if (threadIdx.x < nc * nc) {
    const int q = threadIdx.x / nc, q2 = threadIdx.x % nc;
    const int lo = min(q, q2), hi = max(q, q2);
    a.kent[E.kbase + threadIdx.x] = red[lo * NCMAX - lo * (lo - 1) / 2 + (hi - lo)];
  }
}

template <int NWAVE, int PHIC = 8, int RED = 8>
size_t wave_lds_bytes(const LocalParams& p) {
  return (size_t(1 + PHIC) * p.sig_cap + p.nu_cap + 128 + 40 + RED * 36 + size_t(p.uni_cap)) * sizeof(double);
}

// Shared plane-buffer region of the wave kernels: one plane buffer a wave,
// or four (one a corner) for the one-wave path, and at least the 6 nu
// scaled transmissibilities.
template <int NWAVE>
int wave_uni_cap(const LocalParams& p) {
  const size_t bufs = NWAVE == 1 ? 4 : NWAVE;
  return int(std::max(size_t(6) * p.nu_cap, bufs * p.plane_cap));
}

template <int NWAVE, int NCMAX, int LMAX, int FULLU = 0, bool MULTI = false>
hipError_t launch_wave_t(const LocalParams& pin, bool adj, hipStream_t s) {
  LocalParams p = pin;
  p.uni_cap = wave_uni_cap<NWAVE>(p);
  const size_t lds = wave_lds_bytes<NWAVE, NCMAX, NWAVE>(p);
  if (lds > 160 * 1024) return hipErrorInvalidConfiguration;
  if (adj && !MULTI && !p.mu_scratch) return hipErrorInvalidValue;
  // MULTI: a fixed grid of as many workgroups as fit the device at once
  // (compute units x workgroups a compute unit by LDS), striding over items
  unsigned grid = unsigned(p.nent);
  if constexpr (MULTI) {
    const int per_cu = std::max(1, std::min<int>(int((160 * 1024) / std::max<size_t>(lds, 1)), 2048 / (NWAVE * 64)));
    grid = unsigned(std::min<long long>(p.nent, 256LL * per_cu));
  }
  if (adj) {
    auto kern = k_wave_adj<NWAVE, NCMAX, LMAX, FULLU, MULTI>;
    if (lds > 64 * 1024)
      (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    hipLaunchKernelGGL(kern, dim3(grid), dim3(NWAVE * 64), lds, s, p);
  } else {
    auto kern = k_wave_fwd<NWAVE, NCMAX, LMAX, FULLU, MULTI>;
    if (lds > 64 * 1024)
      (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    hipLaunchKernelGGL(kern, dim3(grid), dim3(NWAVE * 64), lds, s, p);
  }
  return hipGetLastError();
}

template <int NWAVE, int NCMAX, int LMAX>
hipError_t launch_tan_t(const LocalParams& pin, hipStream_t s) {
  LocalParams p = pin;
  p.uni_cap = int(std::max(size_t(6) * p.nu_cap, size_t(NWAVE) * p.plane_cap));
  const size_t lds = wave_lds_bytes<NWAVE>(p) + (size_t(9) * p.sig_cap) * sizeof(double);
  if (lds > 160 * 1024) return hipErrorInvalidConfiguration;
  if (!p.dm || !p.dpval) return hipErrorInvalidValue;
  auto kern = k_wave_tan<NWAVE, NCMAX, LMAX>;
  if (lds > 64 * 1024)
    (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  hipLaunchKernelGGL(kern, dim3(p.nent), dim3(NWAVE * 64), lds, s, p);
  return hipGetLastError();
}

}  // namespace

bool wave_path_fits(const LocalParams& p) {
  return p.lane_cap <= 64 && p.col_cap <= 7 && p.nc_cap <= 8;
}

hipError_t launch_wave_local(const LocalParams& p, bool adj, hipStream_t s) {
  if (p.nent == 0) return hipSuccess;
  if (!wave_path_fits(p)) return hipErrorInvalidConfiguration;
  // four waves a workgroup; dual blocks (8 corners) give each wave two;
  // faces (one cell a lane, four corners) run their corners in one wave
  if (p.nc_cap <= 4) {
    if (p.col_cap <= 1) return launch_wave_t<1, 4, 1>(p, adj, s);
    if (p.col_cap <= 3) return launch_wave_t<4, 4, 3>(p, adj, s);
    return launch_wave_t<4, 4, 7>(p, adj, s);
  }
  if (p.col_cap <= 1) return launch_wave_t<4, 8, 1>(p, adj, s);
  if (p.col_cap <= 3) return launch_wave_t<4, 8, 3>(p, adj, s);
  return launch_wave_t<4, 8, 7>(p, adj, s);
}

// Class of the wave launch launch_wave_local would make for p's caps.
int wave_class(const LocalParams& p) {
  if (p.nc_cap <= 4) {
    if (p.col_cap <= 1) return kClassWave441;
    if (p.col_cap <= 3) return kClassWave443;
    return kClassWave447;
  }
  if (p.col_cap <= 1) return kClassWave481;
  if (p.col_cap <= 3) return kClassWave483;
  return kClassWave487;
}

int wave_class_uni_cap(const LocalParams& p, int klass) {
  const bool one_wave = klass == kClassWave441 || klass == kClassFaces3 || klass == kClassFaces7;
  return one_wave ? wave_uni_cap<1>(p) : wave_uni_cap<4>(p);
}

hipError_t launch_wave_multi(const LocalParams& p, int klass, bool adj, hipStream_t s) {
  switch (klass) {
    case kClassWave441: return launch_wave_t<1, 4, 1, 0, true>(p, adj, s);
    case kClassWave443: return launch_wave_t<4, 4, 3, 0, true>(p, adj, s);
    case kClassWave447: return launch_wave_t<4, 4, 7, 0, true>(p, adj, s);
    case kClassWave481: return launch_wave_t<4, 8, 1, 0, true>(p, adj, s);
    case kClassWave483: return launch_wave_t<4, 8, 3, 0, true>(p, adj, s);
    case kClassWave487: return launch_wave_t<4, 8, 7, 0, true>(p, adj, s);
    case kClassFull3: return launch_wave_t<4, 8, 3, 3, true>(p, adj, s);
    case kClassFull7: return launch_wave_t<4, 8, 7, 7, true>(p, adj, s);
    case kClassFaces3: return launch_wave_t<1, 4, 1, faces_code(3), true>(p, adj, s);
    case kClassFaces7: return launch_wave_t<1, 4, 1, faces_code(7), true>(p, adj, s);
    default: return hipErrorInvalidConfiguration;
  }
}

hipError_t launch_wave_full(const LocalParams& p, int u, bool adj, hipStream_t s) {
  if (p.nent == 0) return hipSuccess;
  if (u == 7) return launch_wave_t<4, 8, 7, 7>(p, adj, s);
  if (u == 3) return launch_wave_t<4, 8, 3, 3>(p, adj, s);
  return hipErrorInvalidConfiguration;
}

hipError_t launch_wave_blocks(const LocalParams& p, int u, hipStream_t s) {
  if (p.nent == 0) return hipSuccess;
  if (!wave_path_fits(p) || p.nc_cap > 8) return hipErrorInvalidConfiguration;
  if (u == 7) return launch_wave_t<4, 8, 7, blocks_code(7)>(p, false, s);
  if (u == 3 && p.col_cap <= 3) return launch_wave_t<4, 8, 3, blocks_code(3)>(p, false, s);
  return hipErrorInvalidConfiguration;
}

hipError_t launch_wave_faces(const LocalParams& p, int u, bool adj, hipStream_t s) {
  if (p.nent == 0) return hipSuccess;
  if (!wave_path_fits(p) || p.nc_cap > 4 || p.col_cap > 1) return hipErrorInvalidConfiguration;
  if (u == 7) return launch_wave_t<1, 4, 1, faces_code(7)>(p, adj, s);
  if (u == 3) return launch_wave_t<1, 4, 1, faces_code(3)>(p, adj, s);
  return hipErrorInvalidConfiguration;
}

hipError_t launch_energy_frozen(const LocalParams& p, hipStream_t s) {
  if (p.nent == 0) return hipSuccess;
  if (p.nc_cap <= 2) {
    hipLaunchKernelGGL(k_energy_frozen<2>, dim3(p.nent), dim3(256), 0, s, p);
  } else if (p.nc_cap <= 4) {
    hipLaunchKernelGGL(k_energy_frozen<4>, dim3(p.nent), dim3(256), 0, s, p);
  } else if (p.nc_cap <= 8) {
    hipLaunchKernelGGL(k_energy_frozen<8>, dim3(p.nent), dim3(256), 0, s, p);
  } else {
    return hipErrorInvalidConfiguration;
  }
  return hipGetLastError();
}

hipError_t launch_wave_tan(const LocalParams& p, hipStream_t s) {
  if (p.nent == 0) return hipSuccess;
  if (!wave_path_fits(p)) return hipErrorInvalidConfiguration;
  if (p.nc_cap <= 4) {
    if (p.col_cap <= 1) return launch_tan_t<4, 4, 1>(p, s);
    if (p.col_cap <= 3) return launch_tan_t<4, 4, 3>(p, s);
    return launch_tan_t<4, 4, 7>(p, s);
  }
  if (p.col_cap <= 1) return launch_tan_t<4, 8, 1>(p, s);
  if (p.col_cap <= 3) return launch_tan_t<4, 8, 3>(p, s);
  return launch_tan_t<4, 8, 7>(p, s);
}

}  // namespace msfv
