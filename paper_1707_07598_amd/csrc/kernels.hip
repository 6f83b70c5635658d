// gfx950 kernels of the adaptive MSFV path.
//
// Forward (Sec. 3.2, eq. multiscaleBasis_step3; eq. reducedPDE; eq. fwdProbRed)
//   k_edge_fwd     one thread per edge entity: the 1-D reduced problem has the
//                  closed form "fraction of cumulative resistance"; also its
//                  energy block.
//   k_local_fwd    one workgroup per face (2 open axes) or dual block (3 open
//                  axes): conductivities of the closed box in LDS, Jacobi-PCG
//                  on the reduced operator for all corners at once (search
//                  directions in LDS, wavefront-shuffle dot products), values
//                  written into the CSR rows of S_k, and the entity's energy
//                  block sum_f T_f dphi_f dphi_f^T over the fluxes it touches.
//   k_kassemble    A_k = S_k^T A S_k as a deterministic gather of energy blocks.
//   k_coarse_pcg   one workgroup per source column: Jacobi-PCG on A_k with
//                  coarse vertex 0 fixed (the potential is fixed at one point).
//   gathers        S_k^T q, D = Rx^T S_k t, u = S_k t.
// Adjoint (Sec. 4.3 eq. sensred and Sec. 4.5, transposed and source-reduced)
//   With lambda_j = A_k^{-1} S_k^T Rx v_j and M = sum_j t_j lambda_j^T, the
//   gradient is sum over basis functions c of the reverse sweep of s_c with
//   load z_c = sum_j (t_jc Rx v_j + lambda_jc q_j) - A y_c,
//   y_c = sum_c' (M + M^T)_{c'c} s_c', plus the flux-derivative term
//   -sum_f dT_f/dm dphi_f^T M dphi_f.  Entities are swept in decreasing
//   dimension; each solves A^E_EE mu_c = z_c|E for its corners, adds
//   -dT_f (dmu_c)(dphi_c) to the flux weight W_f of every flux it touches,
//   and pushes T_f (mu_c + dy_c) onto its Dirichlet neighbours, which belong
//   to the entity of next lower dimension.  k_gfinal turns flux weights into
//   g_i = sum_{f ni i} dT_f/dm_i W_f.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>

#include "kernels.hpp"

namespace msfv {

namespace {

constexpr int kWave = 64;

__device__ __forceinline__ double harm(double a, double b) { return 2.0 * a * b / (a + b); }
// d/dm_a of the harmonic transmissibility for sigma = exp(m)
__device__ __forceinline__ double dharm(double a, double b) {
  double s = a + b;
  return 2.0 * a * b * b / (s * s);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Sum NV values over the workgroup; every thread receives the totals.  The
// butterfly is commutative-exact, so all lanes agree bit for bit, and waves
// are summed in a fixed order: results are deterministic.
template <int NW, int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], int nv, double* red) {
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
#pragma unroll
  for (int i = 0; i < NV; ++i)
    if (i < nv) v[i] = wave_sum(v[i]);
  if (NW == 1) return;
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i)
      if (i < nv) red[wid * NV + i] = v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    if (i < nv) {
      double s = 0.0;
      for (int w = 0; w < NW; ++w) s += red[w * NV + i];
      v[i] = s;
    }
  }
}

__device__ __forceinline__ double p_lookup(const int* prow, const int* pcol, const double* pval,
                                           int gid, int vid) {
  const int a = prow[gid], b = prow[gid + 1];
  double v = 0.0;
  for (int e = a; e < b; ++e)
    if (pcol[e] == vid) v = pval[e];
  return v;
}

// Per own cell the thread keeps only its geometry and diagonal; the
// transmissibilities live in LDS (tp: the +k flux of every own cell, zero
// where there is none), so a thread's state stays in registers.
struct CellGeo {
  int u;      // own-cell index, -1 for an unused slot
  int gid;    // global cell id
  int ci;     // closure index
  int gc[3];  // global coordinates
  int fmask;  // bit d = 2k+plus: a flux of the reduced operator exists in direction d
  int umask;  // bit d: that neighbour is an own cell (else a Dirichlet cell)
  double diag;
  double dinv;
};

__device__ __forceinline__ int gstride_of(const GridInfo& g, int k) {
  return k == 0 ? 1 : (k == 1 ? g.s1 : g.s2);
}

__device__ __forceinline__ int ustride_of(const EntDesc& E, int k) {
  return k == 0 ? 1 : (k == 1 ? E.uext[0] : E.uext[0] * E.uext[1]);
}

__device__ __forceinline__ int cstride_of(const EntDesc& E, int k) {
  return k == 0 ? 1 : (k == 1 ? E.cext[0] : E.cext[0] * E.cext[1]);
}

// Neighbour geometry of own cell u from the closure conductivities in LDS;
// writes the cell's +k transmissibilities to tp[k * nu + u].
__device__ void cell_setup(const EntDesc& E, const GridInfo& g, const double* sig, int u,
                           CellGeo& c, double* tp) {
  c.u = u;
  const int ux = u % E.uext[0];
  const int t = u / E.uext[0];
  const int uy = t % E.uext[1];
  const int uz = t / E.uext[1];
  c.gc[0] = E.ulo[0] + ux;
  c.gc[1] = E.ulo[1] + uy;
  c.gc[2] = E.ulo[2] + uz;
  c.gid = c.gc[0] + g.s1 * c.gc[1] + g.s2 * c.gc[2];
  const int l[3] = {c.gc[0] - E.clo[0], c.gc[1] - E.clo[1], c.gc[2] - E.clo[2]};
  const int cs[3] = {1, E.cext[0], E.cext[0] * E.cext[1]};
  const int uc[3] = {ux, uy, uz};
  const int lc = l[0] + cs[1] * l[1] + cs[2] * l[2];
  c.ci = lc;
  const double s0 = sig[lc];
  double diag = 0.0;
  c.fmask = 0;
  c.umask = 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
#pragma unroll
    for (int pl = 0; pl < 2; ++pl) {
      const int d = 2 * k + pl;
      if (pl) tp[k * E.nu + u] = 0.0;
      if (!((E.open_mask >> k) & 1)) continue;
      const int step = pl ? 1 : -1;
      const int lk = l[k] + step;
      if (lk < 0 || lk >= E.cext[k]) continue;  // outside the closure = outside the domain
      const double tt = harm(s0, sig[lc + step * cs[k]]);
      if (pl) tp[k * E.nu + u] = tt;
      diag += tt;
      c.fmask |= 1 << d;
      const int uk = uc[k] + step;
      if (uk >= 0 && uk < E.uext[k]) c.umask |= 1 << d;
    }
  }
  c.diag = diag;
  c.dinv = diag > 0.0 ? 1.0 / diag : 0.0;
}

// Transmissibility of the flux of cell c in direction d (which must exist):
// the cell's own +k entry, the -k neighbour's +k entry, or, towards a
// Dirichlet cell on the lower side, the harmonic mean from the closure
// conductivities.  The -k entry of an own neighbour is written by another
// thread: read it only after the workgroup barrier that follows the setup.
__device__ __forceinline__ double cell_T(const EntDesc& E, const CellGeo& c, int d, const double* sig,
                                         const double* tp) {
  const int k = d >> 1;
  if (d & 1) return tp[k * E.nu + c.u];
  if ((c.umask >> d) & 1) return tp[k * E.nu + c.u - ustride_of(E, k)];
  return harm(sig[c.ci], sig[c.ci - cstride_of(E, k)]);
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

// Jacobi-PCG on A^E_EE for ncp right-hand sides at once.  Search directions
// live in LDS (pb[c*nu + u]); x, r and p for the thread's own cells live in
// registers.  Stops when ||r_c|| <= rtol ||b_c|| for every column.
// With a start vector x0 the iteration starts from r = b - A x0; the stop
// test stays relative to b.
template <int BLOCK, int CPT, int NCP>
__device__ int local_pcg(const EntDesc& E, const CellGeo (&cg)[CPT], const double* tp, int ncp,
                         const double (&b)[CPT][NCP], double (&x)[CPT][NCP], double* pb,
                         double* redA, double* redB, double tol2, int maxit, bool* ok,
                         const double (*x0)[CPT][NCP] = nullptr, double* res2 = nullptr) {
  constexpr int NW = BLOCK / kWave;
  const int nu = E.nu;
  double r[CPT][NCP], pv[CPT][NCP];
  double sums[2 * NCP];
  double bb[NCP], rz[NCP];
  bool done = true;
  if (!x0) {
#pragma unroll
    for (int c = 0; c < 2 * NCP; ++c) sums[c] = 0.0;
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
#pragma unroll
      for (int c = 0; c < NCP; ++c) {
        x[j][c] = 0.0;
        r[j][c] = b[j][c];
        pv[j][c] = r[j][c] * cg[j].dinv;
        if (cg[j].u >= 0 && c < ncp) {
          sums[c] += b[j][c] * b[j][c];
          sums[NCP + c] += r[j][c] * pv[j][c];
          pb[c * nu + cg[j].u] = pv[j][c];
        }
      }
    }
    block_sum<NW, 2 * NCP>(sums, 2 * NCP, redA);
#pragma unroll
    for (int c = 0; c < NCP; ++c) {
      bb[c] = sums[c];
      rz[c] = sums[NCP + c];
      if (c < ncp && bb[c] > 0.0) done = false;
    }
  } else {
    // ||b|| and x0 in LDS, then r = b - A x0 through the neighbours' x0
    double b2[NCP];
#pragma unroll
    for (int c = 0; c < NCP; ++c) b2[c] = 0.0;
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
#pragma unroll
      for (int c = 0; c < NCP; ++c) {
        x[j][c] = (*x0)[j][c];
        if (cg[j].u >= 0 && c < ncp) {
          b2[c] += b[j][c] * b[j][c];
          pb[c * nu + cg[j].u] = x[j][c];
        }
      }
    }
    block_sum<NW, NCP>(b2, ncp, redA);
    __syncthreads();  // x0 visible to the workgroup
#pragma unroll
    for (int c = 0; c < 2 * NCP; ++c) sums[c] = 0.0;
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
#pragma unroll
      for (int c = 0; c < NCP; ++c) {
        r[j][c] = 0.0;
        pv[j][c] = 0.0;
      }
      if (cg[j].u < 0) continue;
#pragma unroll
      for (int c = 0; c < NCP; ++c) r[j][c] = b[j][c] - cg[j].diag * x[j][c];
#pragma unroll
      for (int d = 0; d < 6; ++d) {
        if (!((cg[j].umask >> d) & 1)) continue;
        const int k = d >> 1;
        const int nb = cg[j].u + ((d & 1) ? ustride_of(E, k) : -ustride_of(E, k));
        const double tt = (d & 1) ? tp[k * nu + cg[j].u] : tp[k * nu + nb];
#pragma unroll
        for (int c = 0; c < NCP; ++c)
          if (c < ncp) r[j][c] += tt * pb[c * nu + nb];
      }
#pragma unroll
      for (int c = 0; c < NCP; ++c) {
        if (c >= ncp) continue;
        pv[j][c] = r[j][c] * cg[j].dinv;
        sums[c] += r[j][c] * r[j][c];
        sums[NCP + c] += r[j][c] * pv[j][c];
      }
    }
    __syncthreads();  // every thread is past its reads of x0
#pragma unroll
    for (int j = 0; j < CPT; ++j)
      if (cg[j].u >= 0)
#pragma unroll
        for (int c = 0; c < NCP; ++c)
          if (c < ncp) pb[c * nu + cg[j].u] = pv[j][c];
    block_sum<NW, 2 * NCP>(sums, 2 * NCP, redB);
#pragma unroll
    for (int c = 0; c < NCP; ++c) {
      bb[c] = b2[c];
      rz[c] = sums[NCP + c];
      if (c < ncp && bb[c] > 0.0 && !(sums[c] <= tol2 * bb[c])) done = false;
    }
  }
  __syncthreads();
  int it = 0;
  *ok = true;
  while (!done) {
    if (it >= maxit) {
      *ok = false;
      break;
    }
    ++it;
    double ap[CPT][NCP];
    double pq[NCP];
#pragma unroll
    for (int c = 0; c < NCP; ++c) pq[c] = 0.0;
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
      if (cg[j].u < 0) continue;
#pragma unroll
      for (int c = 0; c < NCP; ++c) ap[j][c] = cg[j].diag * pv[j][c];
#pragma unroll
      for (int d = 0; d < 6; ++d) {
        if (!((cg[j].umask >> d) & 1)) continue;
        const int k = d >> 1;
        const int nb = cg[j].u + ((d & 1) ? ustride_of(E, k) : -ustride_of(E, k));
        const double tt = (d & 1) ? tp[k * nu + cg[j].u] : tp[k * nu + nb];
#pragma unroll
        for (int c = 0; c < NCP; ++c)
          if (c < ncp) ap[j][c] -= tt * pb[c * nu + nb];
      }
#pragma unroll
      for (int c = 0; c < NCP; ++c)
        if (c < ncp) pq[c] += pv[j][c] * ap[j][c];
    }
    block_sum<NW, NCP>(pq, ncp, redA);
    double alpha[NCP];
#pragma unroll
    for (int c = 0; c < NCP; ++c) alpha[c] = (c < ncp && pq[c] != 0.0) ? rz[c] / pq[c] : 0.0;
#pragma unroll
    for (int c = 0; c < 2 * NCP; ++c) sums[c] = 0.0;
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
      if (cg[j].u < 0) continue;
#pragma unroll
      for (int c = 0; c < NCP; ++c) {
        if (c >= ncp) continue;
        x[j][c] += alpha[c] * pv[j][c];
        r[j][c] -= alpha[c] * ap[j][c];
        const double z = r[j][c] * cg[j].dinv;
        sums[c] += r[j][c] * r[j][c];
        sums[NCP + c] += r[j][c] * z;
      }
    }
    block_sum<NW, 2 * NCP>(sums, 2 * NCP, redB);
    bool conv = true;
    bool bad = false;
#pragma unroll
    for (int c = 0; c < NCP; ++c) {
      if (c >= ncp) continue;
      if (!(sums[c] <= tol2 * bb[c])) conv = false;
      if (sums[c] != sums[c]) bad = true;
    }
    if (conv) break;
    if (bad) {
      *ok = false;
      break;
    }
    double beta[NCP];
#pragma unroll
    for (int c = 0; c < NCP; ++c) {
      beta[c] = (c < ncp && rz[c] != 0.0) ? sums[NCP + c] / rz[c] : 0.0;
      rz[c] = sums[NCP + c];
    }
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
      if (cg[j].u < 0) continue;
#pragma unroll
      for (int c = 0; c < NCP; ++c) {
        if (c >= ncp) continue;
        pv[j][c] = r[j][c] * cg[j].dinv + beta[c] * pv[j][c];
        pb[c * nu + cg[j].u] = pv[j][c];
      }
    }
    __syncthreads();
  }
  if (res2) {
    // (||r|| / ||b||)^2 of the worst column: sums holds the last r.r
    double m2 = 0.0;
#pragma unroll
    for (int c = 0; c < NCP; ++c)
      if (c < ncp && bb[c] > 0.0) {
        double q = sums[c] / bb[c];
        if (!(q >= 0.0)) q = __builtin_huge_val();
        m2 = fmax(m2, q);
      }
    *res2 = m2;
  }
  return it;
}

// Start value of corner c's local solution at an own cell with entity
// coordinates own[] (an entity bounded by vertex planes on each of its open
// axes): the transfinite (Gordon-Hall) interpolation of the corner's values
// on the closure boundary, i.e. the sum over the non-empty sets S of open
// axes of (-1)^(|S|+1) times the blend, along the axes of S, between the two
// planes of each (index coordinates: planes at 0 and U+1), of the values
// with the other coordinates at the cell's own.
__device__ double coons_value(const EntDesc& E, const GridInfo& g, const int* prow, const int* pcol,
                              const double* pval, const int (&own)[3], int vid) {
  int axes[3], na = 0;
#pragma unroll
  for (int k = 0; k < 3; ++k)
    if ((E.open_mask >> k) & 1) axes[na++] = k;
  double sum = 0.0;
  for (int S = 1; S < (1 << na); ++S) {
    const int sz = __popc(S);
    const double sign = (sz & 1) ? 1.0 : -1.0;
    for (int t = 0; t < (1 << sz); ++t) {
      int pos[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) pos[k] = ((E.open_mask >> k) & 1) ? own[k] + 1 : 0;
      double wgt = 1.0;
      int bit = 0;
      for (int q = 0; q < na; ++q) {
        if (!((S >> q) & 1)) continue;
        const int k = axes[q];
        const int side = (t >> bit) & 1;
        ++bit;
        const int n1 = E.uext[k] + 1;
        const double xi = double(own[k] + 1) / n1;
        wgt *= side ? xi : 1.0 - xi;
        pos[k] = side ? n1 : 0;
      }
      const int gid = (E.clo[0] + pos[0]) + g.s1 * (E.clo[1] + pos[1]) + g.s2 * (E.clo[2] + pos[2]);
      sum += sign * wgt * p_lookup(prow, pcol, pval, gid, vid);
    }
  }
  return sum;
}

template <int BLOCK, int CPT>
__device__ void load_closure_sigma(const EntDesc& E, const GridInfo& g, const double* sigma,
                                   double* sig) {
  // sigma = exp(m) of the call's model, formed once per cell by the model copy
  const int ncl = E.cext[0] * E.cext[1] * E.cext[2];
  for (int i = threadIdx.x; i < ncl; i += BLOCK) {
    const int lx = i % E.cext[0];
    const int t = i / E.cext[0];
    const int ly = t % E.cext[1];
    const int lz = t / E.cext[1];
    const int gid = (E.clo[0] + lx) + g.s1 * (E.clo[1] + ly) + g.s2 * (E.clo[2] + lz);
    sig[i] = sigma[gid];
  }
}

// ---------------------------------------------------------------------------
// forward: faces and dual blocks
// ---------------------------------------------------------------------------
template <int BLOCK, int CPT, int NCP>
__device__ __forceinline__ void local_fwd_body(const LocalParams& a, int eid, double* lds) {
  constexpr int NW = BLOCK / kWave;
  const EntDesc& E = a.ents[eid];
  double* sig = lds;
  double* pb = sig + a.sig_cap;
  double* redA = pb + NCP * a.nu_cap;
  double* redB = redA + NW * 40;
  double* tp = redB + NW * 40;  // 3 * nu_cap
  load_closure_sigma<BLOCK, CPT>(E, a.g, a.sig, sig);
  __syncthreads();
  CellGeo cg[CPT];
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    const int u = threadIdx.x + j * BLOCK;
    if (u < E.nu)
      cell_setup(E, a.g, sig, u, cg[j], tp);
    else
      cg[j].u = -1;
  }
  const double tol2 = a.rtol * a.rtol;
  int itmax = 0;
  unsigned long long work = 0;
  bool all_ok = true;
  double resmax = 0.0;
  // faces (and 2-D dual blocks) bounded by vertex planes on both open axes
  // start their solves from the interpolation of the boundary values (8
  // lookups a cell; for 15^3 dual blocks the 26 lookups a cell cost more
  // than the 18 % of CG work they saved: block forward 16.1 -> 18.6 ms at
  // n = 156, r = 16)
  const bool guess = E.bounded_mask == E.open_mask && __popc(E.open_mask) == 2;
  for (int c0 = 0; c0 < E.nc; c0 += NCP) {
    const int ncp = min(NCP, E.nc - c0);
    double x[CPT][NCP];
    if (a.prescribe) {
#pragma unroll
      for (int j = 0; j < CPT; ++j)
#pragma unroll
        for (int c = 0; c < NCP; ++c)
          x[j][c] = (cg[j].u >= 0 && c < ncp) ? lagrange_value(E, cg[j].gc, c0 + c) : 0.0;
    } else {
      double b[CPT][NCP];
#pragma unroll
      for (int j = 0; j < CPT; ++j) {
#pragma unroll
        for (int c = 0; c < NCP; ++c) b[j][c] = 0.0;
        if (cg[j].u < 0) continue;
#pragma unroll
        for (int d = 0; d < 6; ++d) {
          if (!((cg[j].fmask >> d) & 1) || ((cg[j].umask >> d) & 1)) continue;
          const int k = d >> 1;
          const int ng = cg[j].gid + ((d & 1) ? gstride_of(a.g, k) : -gstride_of(a.g, k));
#pragma unroll
          for (int c = 0; c < NCP; ++c)
            if (c < ncp) b[j][c] += cell_T(E, cg[j], d, sig, tp) * p_lookup(a.prow, a.pcol, a.pval, ng, E.vid[c0 + c]);
        }
      }
      __syncthreads();  // previous pass finished with the LDS buffers
      bool ok = true;
      int it;
      double res2 = 0.0;
      if (guess) {
        // start from the interpolation of the boundary values
        double x0[CPT][NCP];
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
#pragma unroll
          for (int c = 0; c < NCP; ++c) x0[j][c] = 0.0;
          if (cg[j].u < 0) continue;
          const int own[3] = {cg[j].gc[0] - E.ulo[0], cg[j].gc[1] - E.ulo[1], cg[j].gc[2] - E.ulo[2]};
#pragma unroll
          for (int c = 0; c < NCP; ++c)
            if (c < ncp) x0[j][c] = coons_value(E, a.g, a.prow, a.pcol, a.pval, own, E.vid[c0 + c]);
        }
        it = local_pcg<BLOCK, CPT, NCP>(E, cg, tp, ncp, b, x, pb, redA, redB, tol2, a.maxit, &ok, &x0, &res2);
      } else {
        it = local_pcg<BLOCK, CPT, NCP>(E, cg, tp, ncp, b, x, pb, redA, redB, tol2, a.maxit, &ok, nullptr,
                                        &res2);
      }
      resmax = fmax(resmax, res2);
      itmax = max(itmax, it);
      all_ok = all_ok && ok;
      work += (unsigned long long)it * E.nu * ncp;
    }
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
      if (cg[j].u < 0) continue;
      const int base = a.prow[cg[j].gid] + c0;
#pragma unroll
      for (int c = 0; c < NCP; ++c)
        if (c < ncp) a.pval[base + c] = x[j][c];
    }
  }
  if (threadIdx.x == 0) {
    if (!all_ok) atomicAdd(a.status + kStLocalNoconv, 1);
    if (a.ent_it) {
      a.ent_it[eid] = itmax;
      if (a.ent_work) a.ent_work[eid] += work;
    }
    if (a.ent_res) a.ent_res[size_t(eid) * 8] = resmax;
  }
  __syncthreads();  // S_k rows of this entity are visible to the workgroup

  // energy block: K_E = sum over touched fluxes T_f dphi_f dphi_f^T
  const int nc = E.nc;
  double kacc[36];
#pragma unroll
  for (int i = 0; i < 36; ++i) kacc[i] = 0.0;
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    if (cg[j].u < 0) continue;
    double pu[8];
    const int base = a.prow[cg[j].gid];
#pragma unroll
    for (int c = 0; c < 8; ++c) pu[c] = c < nc ? a.pval[base + c] : 0.0;
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      if (!((cg[j].fmask >> d) & 1)) continue;
      const bool own = (cg[j].umask >> d) & 1;
      if (!(d & 1) && own) continue;  // counted from the lower own cell
      const int k = d >> 1;
      const int ng = cg[j].gid + ((d & 1) ? gstride_of(a.g, k) : -gstride_of(a.g, k));
      double dp[8];
      const int nbase = a.prow[ng];
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        if (c >= nc) {
          dp[c] = 0.0;
          continue;
        }
        const double pn = own ? a.pval[nbase + c] : p_lookup(a.prow, a.pcol, a.pval, ng, E.vid[c]);
        dp[c] = pu[c] - pn;
      }
      const double tt = cell_T(E, cg[j], d, sig, tp);
      int q = 0;
#pragma unroll
      for (int c = 0; c < 8; ++c)
#pragma unroll
        for (int c2 = c; c2 < 8; ++c2) {
          kacc[q] += tt * dp[c] * dp[c2];
          ++q;
        }
    }
  }
  __syncthreads();
  block_sum<NW, 36>(kacc, 36, redA);
  if (threadIdx.x == 0) {
    int q = 0;
    for (int c = 0; c < 8; ++c)
      for (int c2 = c; c2 < 8; ++c2) {
        if (c < nc && c2 < nc) {
          a.kent[E.kbase + c * nc + c2] = kacc[q];
          a.kent[E.kbase + c2 * nc + c] = kacc[q];
        }
        ++q;
      }
  }
}

template <int BLOCK, int CPT, int NCP, bool MULTI = false>
__global__ __launch_bounds__(BLOCK) void k_local_fwd(LocalParams a) {
  extern __shared__ double lds[];
  if constexpr (MULTI) {
    for (int it = blockIdx.x; it < a.nent; it += gridDim.x) {
      const int2 w = a.items[it];
      local_fwd_body<BLOCK, CPT, NCP>(a.multi[w.x], w.y, lds);
      __syncthreads();  // the next item reuses the LDS tables
    }
  } else {
    local_fwd_body<BLOCK, CPT, NCP>(a, ent_index(a), lds);
  }
}

// ---------------------------------------------------------------------------
// tangent (forward-mode J dm): faces and dual blocks that do not fit one
// wavefront.  For each corner c, A^E_UU dphi_c = -(dA^E phi_c)_U -
// A^E_UB dphi_c|_B (Sec. 4.5 differentiated along dm): the load is
// -sum over the entity's fluxes at an own cell of dT_f (phi_c(i) - phi_c(n))
// plus, towards Dirichlet neighbours, T_f dphi_c(n) from the lower entities'
// tangents already in dS.  Then the tangent energy block dK_E = sum over the
// touched fluxes of dT dphi dphi^T + T (d(dphi) dphi^T + dphi d(dphi)^T).
// Prescribed (Lagrange) entities have dphi = 0 and only the dT term.
// ---------------------------------------------------------------------------
template <int BLOCK, int CPT, int NCP>
__device__ __forceinline__ void local_tan_body(const LocalParams& a, int eid, double* lds) {
  constexpr int NW = BLOCK / kWave;
  const EntDesc& E = a.ents[eid];
  double* sig = lds;
  double* pb = sig + a.sig_cap;
  double* redA = pb + NCP * a.nu_cap;
  double* redB = redA + NW * 40;
  double* tp = redB + NW * 40;  // 3 * nu_cap
  load_closure_sigma<BLOCK, CPT>(E, a.g, a.sig, sig);
  __syncthreads();
  CellGeo cg[CPT];
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    const int u = threadIdx.x + j * BLOCK;
    if (u < E.nu)
      cell_setup(E, a.g, sig, u, cg[j], tp);
    else
      cg[j].u = -1;
  }
  __syncthreads();  // every cell's +k transmissibility is in tp
  // dT of the flux of cell j in direction d (dm of the cell and of its neighbour)
  auto dTf = [&](const CellGeo& c, int d) {
    const int k = d >> 1;
    const int ng = c.gid + ((d & 1) ? gstride_of(a.g, k) : -gstride_of(a.g, k));
    const int cn = c.ci + ((d & 1) ? cstride_of(E, k) : -cstride_of(E, k));
    const double si = sig[c.ci], sn = sig[cn];
    return dharm(si, sn) * a.dm[c.gid] + dharm(sn, si) * a.dm[ng];
  };
  const double tol2 = a.rtol * a.rtol;
  bool all_ok = true;
  for (int c0 = 0; c0 < E.nc; c0 += NCP) {
    const int ncp = min(NCP, E.nc - c0);
    double x[CPT][NCP];
    if (a.prescribe) {
#pragma unroll
      for (int j = 0; j < CPT; ++j)
#pragma unroll
        for (int c = 0; c < NCP; ++c) x[j][c] = 0.0;
    } else {
      double b[CPT][NCP];
#pragma unroll
      for (int j = 0; j < CPT; ++j) {
#pragma unroll
        for (int c = 0; c < NCP; ++c) b[j][c] = 0.0;
        if (cg[j].u < 0) continue;
        const int base = a.prow[cg[j].gid] + c0;
#pragma unroll
        for (int d = 0; d < 6; ++d) {
          if (!((cg[j].fmask >> d) & 1)) continue;
          const bool own = (cg[j].umask >> d) & 1;
          const int k = d >> 1;
          const int ng = cg[j].gid + ((d & 1) ? gstride_of(a.g, k) : -gstride_of(a.g, k));
          const double dt = dTf(cg[j], d);
          const double tt = cell_T(E, cg[j], d, sig, tp);
#pragma unroll
          for (int c = 0; c < NCP; ++c) {
            if (c >= ncp) continue;
            const int vid = E.vid[c0 + c];
            const double pn = own ? a.pval[a.prow[ng] + c0 + c] : p_lookup(a.prow, a.pcol, a.pval, ng, vid);
            b[j][c] -= dt * (a.pval[base + c] - pn);
            if (!own) b[j][c] += tt * p_lookup(a.prow, a.pcol, a.dpval, ng, vid);
          }
        }
      }
      __syncthreads();  // previous pass finished with the LDS buffers
      bool ok = true;
      (void)local_pcg<BLOCK, CPT, NCP>(E, cg, tp, ncp, b, x, pb, redA, redB, tol2, a.maxit, &ok);
      all_ok = all_ok && ok;
    }
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
      if (cg[j].u < 0) continue;
      const int base = a.prow[cg[j].gid] + c0;
#pragma unroll
      for (int c = 0; c < NCP; ++c)
        if (c < ncp) a.dpval[base + c] = x[j][c];
    }
  }
  if (threadIdx.x == 0 && !all_ok) atomicAdd(a.status + kStLocalNoconv, 1);
  __syncthreads();  // the tangent rows of this entity are visible to the workgroup

  const int nc = E.nc;
  double kacc[36];  // upper triangle (dK_E is symmetric)
#pragma unroll
  for (int i = 0; i < 36; ++i) kacc[i] = 0.0;
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    if (cg[j].u < 0) continue;
    double pu[8], du[8];
    const int base = a.prow[cg[j].gid];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      pu[c] = c < nc ? a.pval[base + c] : 0.0;
      du[c] = c < nc ? a.dpval[base + c] : 0.0;
    }
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      if (!((cg[j].fmask >> d) & 1)) continue;
      const bool own = (cg[j].umask >> d) & 1;
      if (!(d & 1) && own) continue;  // counted from the lower own cell
      const int k = d >> 1;
      const int ng = cg[j].gid + ((d & 1) ? gstride_of(a.g, k) : -gstride_of(a.g, k));
      double dp[8], ddp[8];
      const int nbase = a.prow[ng];
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        if (c >= nc) {
          dp[c] = ddp[c] = 0.0;
          continue;
        }
        const double pn = own ? a.pval[nbase + c] : p_lookup(a.prow, a.pcol, a.pval, ng, E.vid[c]);
        const double dn = own ? a.dpval[nbase + c] : p_lookup(a.prow, a.pcol, a.dpval, ng, E.vid[c]);
        dp[c] = pu[c] - pn;
        ddp[c] = du[c] - dn;
      }
      const double tt = cell_T(E, cg[j], d, sig, tp);
      const double dt = dTf(cg[j], d);
      int q = 0;
#pragma unroll
      for (int c = 0; c < 8; ++c)
#pragma unroll
        for (int c2 = c; c2 < 8; ++c2) {
          kacc[q] += dt * dp[c] * dp[c2] + tt * (ddp[c] * dp[c2] + dp[c] * ddp[c2]);
          ++q;
        }
    }
  }
  __syncthreads();
  block_sum<NW, 36>(kacc, 36, redA);
  if (threadIdx.x == 0) {
    int q = 0;
    for (int c = 0; c < 8; ++c)
      for (int c2 = c; c2 < 8; ++c2) {
        if (c < nc && c2 < nc) {
          a.kent[E.kbase + c * nc + c2] = kacc[q];
          a.kent[E.kbase + c2 * nc + c] = kacc[q];
        }
        ++q;
      }
  }
}

template <int BLOCK, int CPT, int NCP>
__global__ __launch_bounds__(BLOCK) void k_local_tan(LocalParams a) {
  extern __shared__ double lds[];
  local_tan_body<BLOCK, CPT, NCP>(a, ent_index(a), lds);
}

// ---------------------------------------------------------------------------
// adjoint: dual blocks and faces
// ---------------------------------------------------------------------------
template <int BLOCK, int CPT, int NCP>
__device__ __forceinline__ void local_adj_body(const LocalParams& a, int eid, double* lds) {
  constexpr int NW = BLOCK / kWave;
  const EntDesc& E = a.ents[eid];
  double* sig = lds;
  double* pb = sig + a.sig_cap;
  double* redA = pb + NCP * a.nu_cap;
  double* redB = redA + NW * 40;
  double* Mm = redB + NW * 40;  // 64
  double* Sm = Mm + 64;         // 64
  double* tp = Sm + 64;         // 3 * nu_cap
  load_closure_sigma<BLOCK, CPT>(E, a.g, a.sig, sig);
  const int nc = E.nc;
  if (threadIdx.x < nc * nc) {
    const int c = threadIdx.x / nc, c2 = threadIdx.x % nc;
    double s = 0.0;
    for (int j = 0; j < a.ns; ++j)
      s += a.t[size_t(j) * a.ncoarse + E.vid[c]] * a.lam[size_t(j) * a.ncoarse + E.vid[c2]];
    Mm[threadIdx.x] = s;
  }
  __syncthreads();
  if (threadIdx.x < nc * nc) {
    const int c = threadIdx.x / nc, c2 = threadIdx.x % nc;
    Sm[threadIdx.x] = Mm[c * nc + c2] + Mm[c2 * nc + c];
  }
  CellGeo cg[CPT];
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    const int u = threadIdx.x + j * BLOCK;
    if (u < E.nu)
      cell_setup(E, a.g, sig, u, cg[j], tp);
    else
      cg[j].u = -1;
  }
  __syncthreads();

  // loads z_c on own cells and the flux-derivative term of the touched fluxes
  double zh[CPT][8];
  double wf[CPT][6];
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
#pragma unroll
    for (int c = 0; c < 8; ++c) zh[j][c] = 0.0;
#pragma unroll
    for (int d = 0; d < 6; ++d) wf[j][d] = 0.0;
    if (cg[j].u < 0) continue;
    const int u = cg[j].u;
    if (E.inbase >= 0) {
      for (int s = 0; s < E.nslot; ++s)
#pragma unroll
        for (int c = 0; c < 8; ++c)
          if (c < nc) zh[j][c] += a.inbuf[E.inbase + (s * nc + c) * E.nu + u];
    }
    for (int e = E.eptr0; e < E.eptr1; ++e)
      if (a.eloc[e] == u)
#pragma unroll
        for (int c = 0; c < 8; ++c)
          if (c < nc) zh[j][c] += a.sload[a.eidx[e] * 8 + c];
    double pu[8];
    const int base = a.prow[cg[j].gid];
#pragma unroll
    for (int c = 0; c < 8; ++c) pu[c] = c < nc ? a.pval[base + c] : 0.0;
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      if (!((cg[j].fmask >> d) & 1)) continue;
      const bool own = (cg[j].umask >> d) & 1;
      const int k = d >> 1;
      const int ng = cg[j].gid + ((d & 1) ? gstride_of(a.g, k) : -gstride_of(a.g, k));
      double dp[8];
      const int nbase = a.prow[ng];
#pragma unroll
      for (int c = 0; c < 8; ++c)
        dp[c] = c < nc ? pu[c] - (own ? a.pval[nbase + c]
                                      : p_lookup(a.prow, a.pcol, a.pval, ng, E.vid[c]))
                       : 0.0;
      // the -(A^E y_c) part of the load is not formed: on own cells it is a
      // combination of the corner bases' local residuals, zero to the local
      // solve tolerance; y_c enters only the pushes below
      double quad = 0.0;
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        if (c >= nc) continue;
        double mq = 0.0;
#pragma unroll
        for (int c2 = 0; c2 < 8; ++c2)
          if (c2 < nc) mq += Mm[c * nc + c2] * dp[c2];
        quad += dp[c] * mq;
      }
      if ((d & 1) || !own) wf[j][d] = -quad;
    }
  }

  // An entity with no electrode loads and no pushes from above (dual blocks
  // off the electrodes) has mu_c = 0 for every corner: the flux weights keep
  // their quadratic part, and one sweep writes the y-part of every corner's
  // pushes, without the corner passes.
  const bool loaded = E.nslot > 0 || E.eptr1 > E.eptr0;
  if (a.solve_adj && !loaded) {
    if (a.push) {
#pragma unroll
      for (int j = 0; j < CPT; ++j) {
        if (cg[j].u < 0) continue;
        const int base = a.prow[cg[j].gid];
#pragma unroll
        for (int d = 0; d < 6; ++d) {
          if (!((cg[j].fmask >> d) & 1) || ((cg[j].umask >> d) & 1)) continue;
          const int te = E.side_ent[d];
          if (te < 0) continue;
          const int k = d >> 1;
          const int ng = cg[j].gid + ((d & 1) ? gstride_of(a.g, k) : -gstride_of(a.g, k));
          double dp[8];
#pragma unroll
          for (int c = 0; c < 8; ++c)
            dp[c] = c < nc ? a.pval[base + c] - p_lookup(a.prow, a.pcol, a.pval, ng, E.vid[c]) : 0.0;
          const EntDesc& R = a.recv[te];
          int gc2[3] = {cg[j].gc[0], cg[j].gc[1], cg[j].gc[2]};
          gc2[k] += (d & 1) ? 1 : -1;
          const int ut = (gc2[0] - R.ulo[0]) + R.uext[0] * ((gc2[1] - R.ulo[1]) + R.uext[1] * (gc2[2] - R.ulo[2]));
          const double tt = cell_T(E, cg[j], d, sig, tp);
#pragma unroll
          for (int c = 0; c < 8; ++c) {
            if (c >= nc) continue;
            int ct = -1;
            for (int q = 0; q < R.nc; ++q)
              if (R.vid[q] == E.vid[c]) ct = q;
            if (ct < 0) continue;
            double dy = 0.0;
#pragma unroll
            for (int c2 = 0; c2 < 8; ++c2)
              if (c2 < nc) dy += Sm[c2 * nc + c] * dp[c2];
            a.outbuf[R.inbase + (E.side_slot[d] * R.nc + ct) * R.nu + ut] = tt * dy;
          }
        }
      }
    }
    if (threadIdx.x == 0 && a.ent_it) a.ent_it[eid] = 0;
    if (threadIdx.x == 0 && a.ent_res) a.ent_res[size_t(eid) * 8] = 0.0;
  } else if (a.solve_adj) {
    const double tol2 = a.rtol * a.rtol;
    int itmax = 0;
    unsigned long long work = 0;
    bool all_ok = true;
    double resmax = 0.0;
    for (int c0 = 0; c0 < nc; c0 += NCP) {
      const int ncp = min(NCP, nc - c0);
      double b[CPT][NCP], x[CPT][NCP];
#pragma unroll
      for (int j = 0; j < CPT; ++j)
#pragma unroll
        for (int c = 0; c < NCP; ++c) b[j][c] = (c < ncp) ? zh[j][c0 + c] : 0.0;
      __syncthreads();
      bool ok = true;
      double res2 = 0.0;
      const int it =
          local_pcg<BLOCK, CPT, NCP>(E, cg, tp, ncp, b, x, pb, redA, redB, tol2, a.maxit, &ok, nullptr, &res2);
      resmax = fmax(resmax, res2);
      itmax = max(itmax, it);
      all_ok = all_ok && ok;
      work += (unsigned long long)it * E.nu * ncp;
      __syncthreads();
#pragma unroll
      for (int j = 0; j < CPT; ++j)
        if (cg[j].u >= 0)
#pragma unroll
          for (int c = 0; c < NCP; ++c)
            if (c < ncp) pb[c * E.nu + cg[j].u] = x[j][c];
      __syncthreads();
      // flux weights and pushes for this pass's corners
#pragma unroll
      for (int j = 0; j < CPT; ++j) {
        if (cg[j].u < 0) continue;
        const int base = a.prow[cg[j].gid];
#pragma unroll
        for (int d = 0; d < 6; ++d) {
          if (!((cg[j].fmask >> d) & 1)) continue;
          const bool own = (cg[j].umask >> d) & 1;
          const int k = d >> 1;
          const int ng = cg[j].gid + ((d & 1) ? gstride_of(a.g, k) : -gstride_of(a.g, k));
          const int nb = cg[j].u + ((d & 1) ? ustride_of(E, k) : -ustride_of(E, k));
          const int nbase = a.prow[ng];
          double dp[8];
#pragma unroll
          for (int c = 0; c < 8; ++c)
            dp[c] = c < nc ? a.pval[base + c] - (own ? a.pval[nbase + c]
                                                     : p_lookup(a.prow, a.pcol, a.pval, ng, E.vid[c]))
                           : 0.0;
          if ((d & 1) || !own) {
            double s = 0.0;
#pragma unroll
            for (int c = 0; c < NCP; ++c) {
              if (c >= ncp) continue;
              const double mun = own ? pb[c * E.nu + nb] : 0.0;
              s += (x[j][c] - mun) * dp[c0 + c];
            }
            wf[j][d] -= s;
          }
          if (!own && a.push) {
            const int te = E.side_ent[d];
            if (te < 0) continue;
            const EntDesc& R = a.recv[te];
            int gc2[3] = {cg[j].gc[0], cg[j].gc[1], cg[j].gc[2]};
            gc2[k] += (d & 1) ? 1 : -1;
            const int ut = (gc2[0] - R.ulo[0]) + R.uext[0] * ((gc2[1] - R.ulo[1]) + R.uext[1] * (gc2[2] - R.ulo[2]));
            const double tt = cell_T(E, cg[j], d, sig, tp);
#pragma unroll
            for (int c = 0; c < NCP; ++c) {
              if (c >= ncp) continue;
              const int vid = E.vid[c0 + c];
              int ct = -1;
              for (int q = 0; q < R.nc; ++q)
                if (R.vid[q] == vid) ct = q;
              if (ct < 0) continue;
              double dy = 0.0;
#pragma unroll
              for (int c2 = 0; c2 < 8; ++c2)
                if (c2 < nc) dy += Sm[c2 * nc + c0 + c] * dp[c2];
              a.outbuf[R.inbase + (E.side_slot[d] * R.nc + ct) * R.nu + ut] = tt * (x[j][c] + dy);
            }
          }
        }
      }
    }
    if (threadIdx.x == 0) {
      if (!all_ok) atomicAdd(a.status + kStLocalNoconv, 1);
      if (a.ent_it) {
        a.ent_it[eid] = itmax;
        if (a.ent_work) a.ent_work[eid] += work;
      }
      if (a.ent_res) a.ent_res[size_t(eid) * 8] = resmax;
    }
  }
  // flux weights of the fluxes this entity owns
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    if (cg[j].u < 0) continue;
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      if (!((cg[j].fmask >> d) & 1)) continue;
      const bool own = (cg[j].umask >> d) & 1;
      if (!(d & 1) && own) continue;
      const int k = d >> 1;
      const int lower = (d & 1) ? cg[j].gid : cg[j].gid - gstride_of(a.g, k);
      const long long N = (long long)a.g.n[0] * a.g.n[1] * a.g.n[2];
      a.W[k * N + lower] = wf[j][d];
    }
  }
}

template <int BLOCK, int CPT, int NCP, bool MULTI = false>
__global__ __launch_bounds__(BLOCK) void k_local_adj(LocalParams a) {
  extern __shared__ double lds[];
  if constexpr (MULTI) {
    for (int it = blockIdx.x; it < a.nent; it += gridDim.x) {
      const int2 w = a.items[it];
      local_adj_body<BLOCK, CPT, NCP>(a.multi[w.x], w.y, lds);
      __syncthreads();  // the next item reuses the LDS tables
    }
  } else {
    local_adj_body<BLOCK, CPT, NCP>(a, ent_index(a), lds);
  }
}

// ---------------------------------------------------------------------------
// edges: closed-form forward, tridiagonal adjoint (one thread per edge)
// ---------------------------------------------------------------------------
constexpr int kMaxLine = 17;  // closure cells along an edge for r <= 16

struct EdgeLine {
  int k, len, base, st, u0;
  double sig[kMaxLine];
  double T[kMaxLine];
};

// sigma = exp(m) of the call's model (formed once per cell by the model copy)
__device__ void edge_line(const EntDesc& E, const GridInfo& g, const double* sigma, EdgeLine& L) {
  L.k = (E.open_mask & 1) ? 0 : ((E.open_mask & 2) ? 1 : 2);
  L.len = E.cext[L.k];
  L.base = E.clo[0] + g.s1 * E.clo[1] + g.s2 * E.clo[2];
  L.st = gstride_of(g, L.k);
  L.u0 = E.ulo[L.k] - E.clo[L.k];
  for (int i = 0; i < L.len; ++i) L.sig[i] = sigma[L.base + i * L.st];
  for (int i = 0; i + 1 < L.len; ++i) L.T[i] = harm(L.sig[i], L.sig[i + 1]);
}

// basis values of the edge's corners at closure position i
__device__ __forceinline__ void edge_phi(const EntDesc& E, const EdgeLine& L, const double* cum,
                                         int lagrange, int i, double* phi) {
  if (E.nc == 1) {
    phi[0] = 1.0;
    return;
  }
  if (lagrange) {
    const double h = L.len - 1;
    phi[0] = (h - i) / h;
    phi[1] = double(i) / h;
  } else {
    const double R = cum[L.len - 1];
    phi[0] = (R - cum[i]) / R;
    phi[1] = cum[i] / R;
  }
}

// The forward and adjoint edge kernels keep an edge's closure line (LM
// cells at most: 9 for coarsening up to 8, 17 up to 16) in registers: every
// loop over the line is unrolled with the edge's own length as a predicate,
// so no array is indexed at run time (indexed so, they would live in scratch
// memory).  T[i]: transmissibility between line cells i and i + 1.
template <int LM>
struct EdgeRow {
  int k, len, base, st, u0;
  double T[LM];
  double cum[LM];  // cumulative resistances: cum[i] = sum_{f < i} 1 / T[f], constant past the line's end
};

template <int LM>
__device__ __forceinline__ void edge_row(const EntDesc& E, const GridInfo& g, const double* sigma,
                                         EdgeRow<LM>& L) {
  L.k = (E.open_mask & 1) ? 0 : ((E.open_mask & 2) ? 1 : 2);
  L.len = E.cext[L.k];
  L.base = E.clo[0] + g.s1 * E.clo[1] + g.s2 * E.clo[2];
  L.st = gstride_of(g, L.k);
  L.u0 = E.ulo[L.k] - E.clo[L.k];
  double sg[LM];
#pragma unroll
  for (int i = 0; i < LM; ++i) sg[i] = i < L.len ? sigma[L.base + i * L.st] : 1.0;
#pragma unroll
  for (int i = 0; i < LM; ++i) L.T[i] = (i + 1 < LM && i + 1 < L.len) ? harm(sg[i], sg[i + 1 < LM ? i + 1 : i]) : 0.0;
  L.cum[0] = 0.0;
#pragma unroll
  for (int i = 0; i + 1 < LM; ++i) L.cum[i + 1] = i + 1 < L.len ? L.cum[i] + 1.0 / L.T[i] : L.cum[i];
}

// basis values of the edge's corners at line position i (i fixed at compile
// time after unrolling)
template <int LM>
__device__ __forceinline__ void edge_phi_at(const EntDesc& E, const EdgeRow<LM>& L, int lagrange, int i,
                                            double* phi) {
  if (E.nc == 1) {
    phi[0] = 1.0;
    phi[1] = 0.0;
    return;
  }
  if (lagrange) {
    const double h = L.len - 1;
    phi[0] = (h - i) / h;
    phi[1] = double(i) / h;
  } else {
    const double R = L.cum[LM - 1];
    phi[0] = (R - L.cum[i]) / R;
    phi[1] = L.cum[i] / R;
  }
}

template <int LM>
__device__ __forceinline__ void edge_fwd_one(const LocalParams& a, int e, int lagrange) {
  const EntDesc& E = a.ents[e];
  EdgeRow<LM> L;
  edge_row<LM>(E, a.g, a.sig, L);
#pragma unroll
  for (int i = 0; i < LM; ++i) {
    if (i < L.u0 || i >= L.u0 + E.nu) continue;
    double phi[2];
    edge_phi_at<LM>(E, L, lagrange, i, phi);
    const int row = a.prow[L.base + i * L.st];
    for (int c = 0; c < E.nc; ++c) a.pval[row + c] = phi[c];
  }
  double k00 = 0.0, k01 = 0.0, k11 = 0.0;
#pragma unroll
  for (int i = 0; i + 1 < LM; ++i) {
    if (i + 1 >= L.len || E.nc == 1) continue;
    double pa[2], pb2[2];
    edge_phi_at<LM>(E, L, lagrange, i, pa);
    edge_phi_at<LM>(E, L, lagrange, i + 1, pb2);
    const double d0 = pa[0] - pb2[0], d1 = pa[1] - pb2[1];
    k00 += L.T[i] * d0 * d0;
    k01 += L.T[i] * d0 * d1;
    k11 += L.T[i] * d1 * d1;
  }
  if (E.nc == 1) {
    a.kent[E.kbase] = 0.0;
  } else {
    a.kent[E.kbase + 0] = k00;
    a.kent[E.kbase + 1] = k01;
    a.kent[E.kbase + 2] = k01;
    a.kent[E.kbase + 3] = k11;
  }
}

template <int LM>
__global__ __launch_bounds__(64) void k_edge_fwd(LocalParams a, int lagrange) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.nent) return;
  edge_fwd_one<LM>(a, e, lagrange);
}

// Tangent of the edge basis along dm (Sec. 4.5, forward mode): with
// cumulative resistances c_i = sum_{f<i} 1/T_f and R = c_last,
// phi_hi = c_i / R, phi_lo = 1 - phi_hi, so dphi_hi = (dc_i R - c_i dR) / R^2
// with dc_i = -sum_{f<i} dT_f / T_f^2.  Strips and Lagrange edges do not depend
// on m.  Also the tangent energy block dK_E = sum_f dT_f dphi dphi^T +
// T_f (d(dphi) dphi^T + dphi d(dphi)^T) over the edge's fluxes.
__global__ void k_edge_tan(LocalParams a, int lagrange) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.nent) return;
  const EntDesc E = a.ents[e];
  EdgeLine L;
  edge_line(E, a.g, a.sig, L);
  double cum[kMaxLine], dcum[kMaxLine], dT[kMaxLine];
  cum[0] = dcum[0] = 0.0;
  for (int i = 0; i + 1 < L.len; ++i) {
    const double da = a.dm[L.base + i * L.st], db = a.dm[L.base + (i + 1) * L.st];
    dT[i] = dharm(L.sig[i], L.sig[i + 1]) * da + dharm(L.sig[i + 1], L.sig[i]) * db;
    cum[i + 1] = cum[i] + 1.0 / L.T[i];
    dcum[i + 1] = dcum[i] - dT[i] / (L.T[i] * L.T[i]);
  }
  const bool fixed = E.nc == 1 || lagrange;
  const double R = cum[L.len - 1], dR = dcum[L.len - 1];
  auto tan = [&](int i, double* d) {
    if (fixed) {
      d[0] = d[1] = 0.0;
      return;
    }
    const double d1 = (dcum[i] * R - cum[i] * dR) / (R * R);
    d[0] = -d1;
    d[1] = d1;
  };
  for (int q = 0; q < E.nu; ++q) {
    const int i = L.u0 + q;
    double d[2];
    tan(i, d);
    const int row = a.prow[L.base + i * L.st];
    for (int c = 0; c < E.nc; ++c) a.dpval[row + c] = d[c];
  }
  if (E.nc == 1) {
    a.kent[E.kbase] = 0.0;
    return;
  }
  double k00 = 0.0, k01 = 0.0, k11 = 0.0;
  for (int i = 0; i + 1 < L.len; ++i) {
    double pa[2], pb[2], da[2], db[2];
    edge_phi(E, L, cum, lagrange, i, pa);
    edge_phi(E, L, cum, lagrange, i + 1, pb);
    tan(i, da);
    tan(i + 1, db);
    const double f0 = pa[0] - pb[0], f1 = pa[1] - pb[1];
    const double g0 = da[0] - db[0], g1 = da[1] - db[1];
    k00 += dT[i] * f0 * f0 + 2.0 * L.T[i] * g0 * f0;
    k01 += dT[i] * f0 * f1 + L.T[i] * (g0 * f1 + f0 * g1);
    k11 += dT[i] * f1 * f1 + 2.0 * L.T[i] * g1 * f1;
  }
  a.kent[E.kbase + 0] = k00;
  a.kent[E.kbase + 1] = k01;
  a.kent[E.kbase + 2] = k01;
  a.kent[E.kbase + 3] = k11;
}

template <int LM>
__device__ __forceinline__ void edge_adj_one(const LocalParams& a, int e, int lagrange) {
  const EntDesc& E = a.ents[e];
  EdgeRow<LM> L;
  edge_row<LM>(E, a.g, a.sig, L);
  const long long N = (long long)a.g.n[0] * a.g.n[1] * a.g.n[2];
  double* Wk = a.W + L.k * N;
  if (E.nc == 1) {  // strip: s = 1 for every m, nothing depends on m
#pragma unroll
    for (int i = 0; i + 1 < LM; ++i)
      if (i + 1 < L.len) Wk[L.base + i * L.st] = 0.0;
    return;
  }
  double M[4] = {0, 0, 0, 0};
  // unrolled: the loads of several sources in flight together (the sums
  // keep their order)
#pragma unroll 8
  for (int j = 0; j < a.ns; ++j) {
    const double t0 = a.t[size_t(j) * a.ncoarse + E.vid[0]], t1 = a.t[size_t(j) * a.ncoarse + E.vid[1]];
    const double l0 = a.lam[size_t(j) * a.ncoarse + E.vid[0]], l1 = a.lam[size_t(j) * a.ncoarse + E.vid[1]];
    M[0] += t0 * l0;
    M[1] += t0 * l1;
    M[2] += t1 * l0;
    M[3] += t1 * l1;
  }
  const double S[4] = {2 * M[0], M[1] + M[2], M[1] + M[2], 2 * M[3]};
  // mu = (A^E_EE)^{-1} z on the own cells (line positions u0 .. u0 + nu - 1;
  // 1 .. len - 2 for a bounded edge): the loads z first, then the Thomas
  // algorithm in place (an M-matrix, no pivoting).  Lagrange edges have no
  // local problem: mu = 0.
  double mu0[LM], mu1[LM];
  const int i0 = L.u0, i1 = L.u0 + E.nu - 1;
#pragma unroll
  for (int i = 0; i < LM; ++i) {
    mu0[i] = mu1[i] = 0.0;
    if (lagrange || i < i0 || i > i1) continue;
    const int q = i - L.u0;
    double l0 = 0.0, l1 = 0.0;
    for (int s = 0; s < E.nslot; ++s) {
      l0 += a.inbuf[E.inbase + (s * 2 + 0) * E.nu + q];
      l1 += a.inbuf[E.inbase + (s * 2 + 1) * E.nu + q];
    }
    for (int ee = E.eptr0; ee < E.eptr1; ++ee)
      if (a.eloc[ee] == q) {
        l0 += a.sload[a.eidx[ee] * 8 + 0];
        l1 += a.sload[a.eidx[ee] * 8 + 1];
      }
    double pu[2], pn[2];
    edge_phi_at<LM>(E, L, lagrange, i, pu);
    // the own cells of a bounded edge have both line neighbours (the
    // clamped positions below only keep the unrolled indices in range)
    const int kLo = i > 0 ? i - 1 : 0, kHi = i + 1 < LM ? i + 1 : LM - 1;
    edge_phi_at<LM>(E, L, lagrange, kLo, pn);
    {
      const double d0 = pu[0] - pn[0], d1 = pu[1] - pn[1];
      l0 -= L.T[kLo] * (S[0] * d0 + S[2] * d1);
      l1 -= L.T[kLo] * (S[1] * d0 + S[3] * d1);
    }
    edge_phi_at<LM>(E, L, lagrange, kHi, pn);
    {
      const double d0 = pu[0] - pn[0], d1 = pu[1] - pn[1];
      l0 -= L.T[i] * (S[0] * d0 + S[2] * d1);
      l1 -= L.T[i] * (S[1] * d0 + S[3] * d1);
    }
    mu0[i] = l0;
    mu1[i] = l1;
  }
  if (!lagrange) {
    double cp[LM];
#pragma unroll
    for (int i = 0; i < LM; ++i) {
      cp[i] = 0.0;
      if (i < i0 || i > i1) continue;
      const int im = i > 0 ? i - 1 : 0;
      const bool first = !(i > 0 && i > i0);
      const double lo = i > 0 ? L.T[im] : 0.0;
      const double hi = i + 1 < L.len ? L.T[i] : 0.0;
      const double diag = lo + hi;
      const double sub = first ? 0.0 : -lo;
      const double den = diag - sub * (first ? 0.0 : cp[im]);
      cp[i] = (i < i1) ? -hi / den : 0.0;
      mu0[i] = (mu0[i] - sub * (first ? 0.0 : mu0[im])) / den;
      mu1[i] = (mu1[i] - sub * (first ? 0.0 : mu1[im])) / den;
    }
#pragma unroll
    for (int i = LM - 2; i >= 0; --i) {
      if (i < i0 || i >= i1) continue;
      mu0[i] -= cp[i] * mu0[i + 1];
      mu1[i] -= cp[i] * mu1[i + 1];
    }
  }
#pragma unroll
  for (int i = 0; i + 1 < LM; ++i) {
    if (i + 1 >= L.len) continue;
    double pa[2], pb2[2];
    edge_phi_at<LM>(E, L, lagrange, i, pa);
    edge_phi_at<LM>(E, L, lagrange, i + 1, pb2);
    const double d0 = pa[0] - pb2[0], d1 = pa[1] - pb2[1];
    const double quad = d0 * (M[0] * d0 + M[1] * d1) + d1 * (M[2] * d0 + M[3] * d1);
    const double w = -((mu0[i] - mu0[i + 1]) * d0 + (mu1[i] - mu1[i + 1]) * d1) - quad;
    Wk[L.base + i * L.st] = w;
  }
}

template <int LM>
__global__ __launch_bounds__(64) void k_edge_adj(LocalParams a, int lagrange) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.nent) return;
  edge_adj_one<LM>(a, e, lagrange);
}

// edges of many problems: one thread an item
template <int LM>
__global__ __launch_bounds__(128) void k_edge_multi(LocalParams a, int adj) {
  const int it = blockIdx.x * blockDim.x + threadIdx.x;
  if (it >= a.nent) return;
  const int2 w = a.items[it];
  const LocalParams& A = a.multi[w.x];
  if (adj)
    edge_adj_one<LM>(A, w.y, A.lagrange);
  else
    edge_fwd_one<LM>(A, w.y, A.lagrange);
}

// ---------------------------------------------------------------------------
// coarse operator, coarse solve, gathers
// ---------------------------------------------------------------------------
__global__ void k_check_finite(const double* m, long long n, int* status) {
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  bool bad = false;
  for (; i < n; i += (long long)gridDim.x * blockDim.x) {
    const double v = m[i];
    if (!isfinite(v)) bad = true;
  }
  if (bad) atomicOr(status + kStNonfinite, 1);
}

// The model of a call: dst = m, sig = exp(m), and the non-finite flag.
__global__ void k_prep_model(double* __restrict__ dst, double* __restrict__ sig,
                             const double* __restrict__ src, long long n, int* status) {
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  bool bad = false;
  for (; i < n; i += (long long)gridDim.x * blockDim.x) {
    const double v = src[i];
    dst[i] = v;
    sig[i] = exp(v);
    if (!isfinite(v)) bad = true;
  }
  if (bad) atomicOr(status + kStNonfinite, 1);
}

__global__ void k_zero_words(unsigned* p, long long n) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

__global__ void k_copy_d(double* __restrict__ dst, const double* __restrict__ src, long long n) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

__global__ void k_set_ones(const int* idx, int n, double* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[idx[i]] = 1.0;
}

__global__ void k_kassemble(const int* kcptr, const int* kcidx, const int* dslot, const double* kent,
                            double* kval, double* kdia, int nnz) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nnz) return;
  double s = 0.0;
  for (int e = kcptr[i]; e < kcptr[i + 1]; ++e) s += kent[kcidx[e]];
  kval[i] = s;
  kdia[dslot[i]] = s;
}

__global__ void k_gather_slots(const int* slot_dst, const int* slot_ptr, const int* ent_pidx,
                               const double* ent_w, const int* ent_col, const double* colw,
                               int colw_ld, const double* pval, double* out, int nslot, int ncol,
                               int nc) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= (long long)nslot * ncol) return;
  const int s = int(t % nslot), j = int(t / nslot);
  double acc = 0.0;
  const int e0 = slot_ptr[s], e1 = slot_ptr[s + 1];
  // the slot's entries four at a time, their loads in flight together
  for (int eb = e0; eb < e1; eb += 4) {
    double w[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = eb + u;
      w[u] = 0.0;
      if (e >= e1) continue;
      w[u] = ent_w[e] * pval[ent_pidx[e]];
      if (colw) w[u] *= colw[size_t(j) * colw_ld + ent_col[e]];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (eb + u < e1) acc += w[u];
  }
  out[slot_dst[s] + size_t(j) * nc] = acc;
}

__global__ void k_data(const int* rptr, const int* rcell, const double* rval, int nr, int ns,
                       const int* prow, const int* pcol, const double* pval, const double* t, int nc,
                       double* D, int accumulate) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= nr * ns) return;
  const int i = tid % nr, j = tid / nr;
  const double* tj = t + size_t(j) * nc;
  double acc = 0.0;
  for (int e = rptr[i]; e < rptr[i + 1]; ++e) {
    const int cell = rcell[e];
    double uval = 0.0;
    for (int q = prow[cell]; q < prow[cell + 1]; ++q) uval += pval[q] * tj[pcol[q]];
    acc += rval[e] * uval;
  }
  if (accumulate)
    D[size_t(j) * nr + i] += acc;
  else
    D[size_t(j) * nr + i] = acc;
}

// tT[v * ldt + j] = t[j * nc + v]: the coarse coefficients vertex by vertex,
// sources contiguous (rows padded to ldt, a multiple of 4, with zeros)
__global__ void k_transpose_t(const double* __restrict__ t, int nc, int ns, int ldt, double* __restrict__ tT) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= (long long)nc * ldt) return;
  const int v = int(i / ldt), j = int(i % ldt);
  tT[i] = j < ns ? t[size_t(j) * nc + v] : 0.0;
}

// u_j = S_k t_j for every source: one cell a thread, its S_k row in
// registers, each source's value stored coalesced across the wave.  The
// coefficients come from the vertex-major copy tT (row v: the ldt values of
// vertex v).  A workgroup's 256 consecutive cells draw on the vertices of at
// most a few vertex rows J of at most two vertex planes K; when they fit the
// box of kProlongK planes x kProlongJ rows (and the box fits the dynamic LDS
// the launch gave), the workgroup stages those rows of tT in LDS with
// contiguous 16-byte loads and gathers from there instead of through the
// vector memory path; otherwise it gathers from tT directly.  Either way the
// sums run in the same order, so u is the same bit for bit.
constexpr int kProlongK = 2, kProlongJ = 3;

__device__ __forceinline__ int wave_min_i(int v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, kWave));
  return v;
}

__global__ __launch_bounds__(256) void k_prolong(const int* __restrict__ prow, const int* __restrict__ pcol,
                                                 const double* __restrict__ pval, const double* __restrict__ tT,
                                                 int ldt, int ns, int ncx, int ncy, int nc, long long ncell,
                                                 int staged, double* __restrict__ u) {
  extern __shared__ double tl[];  // staged: kProlongK * kProlongJ * ncx vertices, ldt + 2 apart
  __shared__ int red[4][4];
  const long long cell = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const bool live = cell < ncell;
  const int a = live ? prow[cell] : 0;
  const int len = live ? prow[cell + 1] - a : 0;
  int col[8];
  double val[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    col[q] = q < len ? pcol[a + q] : 0;
    val[q] = q < len ? pval[a + q] : 0.0;
  }
  bool boxed = false;
  int j0 = 0, k0 = 0;
  if (staged) {
    // (min J, -max J, min K, -max K) over the workgroup's columns
    const int pl = ncx * ncy;
    int m4[4] = {INT_MAX, INT_MAX, INT_MAX, INT_MAX};
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (q >= len) continue;
      const int K = col[q] / pl, J = (col[q] - K * pl) / ncx;
      m4[0] = min(m4[0], J);
      m4[1] = min(m4[1], -J);
      m4[2] = min(m4[2], K);
      m4[3] = min(m4[3], -K);
    }
    const int wid = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int i = 0; i < 4; ++i) m4[i] = wave_min_i(m4[i]);
    if (lane == 0) {
#pragma unroll
      for (int i = 0; i < 4; ++i) red[wid][i] = m4[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i) m4[i] = min(min(red[0][i], red[1][i]), min(red[2][i], red[3][i]));
    j0 = m4[0];
    k0 = m4[2];
    // no live column at all (m4 = INT_MAX): nothing to stage, nothing to gather
    boxed = m4[0] != INT_MAX && -m4[1] - j0 < kProlongJ && -m4[3] - k0 < kProlongK;
    if (boxed) {
      // vertex w of the box at tl + w * (ldt + 2): the pad spreads the
      // vertices a wave reads at once over the LDS banks (ldt is a multiple
      // of 4, so every vertex stays 16-byte aligned)
      const int half = ncx * ldt / 2, hv = ldt / 2;
      for (int e = threadIdx.x; e < kProlongK * kProlongJ * half; e += 256) {
        const int b = e / half, o = e - b * half;
        const int kk = b / kProlongJ, jj = b - kk * kProlongJ;
        const int J = j0 + jj, K = k0 + kk;
        if (J >= ncy || (K * ncy + J + 1) * ncx > nc) continue;  // past the grid: never read
        const double2* src = reinterpret_cast<const double2*>(tT + size_t(K * ncy + J) * ncx * ldt);
        const int w = b * ncx + o / hv, h = o - (o / hv) * hv;
        reinterpret_cast<double2*>(tl + size_t(w) * (ldt + 2))[h] = src[o];
      }
      __syncthreads();
    }
  }
  if (!live) return;
  // position of each column's coefficients (LDS box or tT)
  const double* base[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    if (q >= len) {
      base[q] = tT;  // not read
    } else if (boxed) {
      const int pl = ncx * ncy;
      const int K = col[q] / pl, r = col[q] - K * pl, J = r / ncx, I = r - J * ncx;
      base[q] = tl + size_t(((K - k0) * kProlongJ + (J - j0)) * ncx + I) * (ldt + 2);
    } else {
      base[q] = tT + size_t(col[q]) * ldt;
    }
  }
  for (int jb = 0; jb < ns; jb += 4) {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (q < len) {
        const double2* tp = reinterpret_cast<const double2*>(base[q] + jb);
        const double2 lo = tp[0], hi = tp[1];
        acc[0] += val[q] * lo.x;
        acc[1] += val[q] * lo.y;
        acc[2] += val[q] * hi.x;
        acc[3] += val[q] * hi.y;
      }
    }
#pragma unroll
    for (int jj = 0; jj < 4; ++jj)
      if (jb + jj < ns) u[size_t(jb + jj) * ncell + cell] = acc[jj];
  }
}

// direct loads at electrode cells: s_c = sum_j t_jc (Rx v_j)(cell) + lambda_jc q_j(cell)
__global__ void k_sload(int nelec, const int* ecell, const int* rptr, const int* ridx,
                        const double* rw, const int* sptr, const int* sidx, const double* sw,
                        const int* prow, const int* pcol, const double* t, const double* lam,
                        const double* v, int nc, int ns, int nr, double* sload) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= nelec * 8) return;
  const int e = tid / 8, c = tid % 8;
  const int cell = ecell[e];
  const int a = prow[cell], len = prow[cell + 1] - a;
  double acc = 0.0;
  if (c < len) {
    const int vid = pcol[a + c];
    const double* tv = t + vid;
    // receivers at the cell (usually one), then the sources in an unrolled
    // loop whose loads are in flight together
    for (int q = rptr[e]; q < rptr[e + 1]; ++q) {
      const double wq = rw[q];
      const double* vq = v + ridx[q];
#pragma unroll 8
      for (int j = 0; j < ns; ++j) acc += tv[size_t(j) * nc] * (wq * vq[size_t(j) * nr]);
    }
    for (int q = sptr[e]; q < sptr[e + 1]; ++q) acc += lam[size_t(sidx[q]) * nc + vid] * sw[q];
  }
  sload[e * 8 + c] = acc;
}

// g_i = sum over the fluxes f of cell i of dT_f/dm_i W_f, with sigma = exp(m)
// precomputed.  One workgroup a span of 256 consecutive cells.  Workgroups go round-robin
// over the eight XCDs (workgroup L to XCD L mod 8), so span = (L mod 8) * spx
// + L / 8 gives XCD x the contiguous spans [x spx, (x+1) spx): the rows and
// planes whose sigma and W a span reads around its own cells (i +- n_x,
// i +- n_x n_y) are then mostly in that XCD's L2, and HBM sees each array
// about once.
__global__ __launch_bounds__(256) void k_gfinal(const double* __restrict__ sig, const double* __restrict__ W,
                                                GridInfo g, int ncell, int spx, double* __restrict__ grad) {
  const int span = int(blockIdx.x % 8u) * spx + int(blockIdx.x / 8u);
  const int i = span * 256 + int(threadIdx.x);
  if (i >= ncell) return;
  const int row = i / g.n[0];
  const int c[3] = {i - row * g.n[0], row % g.n[1], row / g.n[1]};
  const double si = sig[i];
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int st = gstride_of(g, k);
    const double* Wk = W + (long long)k * ncell;
    if (c[k] + 1 < g.n[k]) acc += dharm(si, sig[i + st]) * Wk[i];
    if (c[k] > 0) acc += dharm(si, sig[i - st]) * Wk[i - st];
  }
  grad[i] = acc;
}

// y_j = (dA/dm . dm) u_j: per cell i, sum over its faces f = (i, n) of
// dT_f (u_j(i) - u_j(n)) with dT_f = dT/dm_i dm_i + dT/dm_n dm_n.
__global__ void k_dAu(const double* m, const double* dm, GridInfo g, long long ncell, int ns,
                      const double* u, double* y) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= ncell) return;
  const int c[3] = {int(i % g.n[0]), int((i / g.n[0]) % g.n[1]), int(i / ((long long)g.n[0] * g.n[1]))};
  const double si = exp(m[i]);
  double dT[6];
  long long nb[6];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int st = gstride_of(g, k);
#pragma unroll
    for (int sd = 0; sd < 2; ++sd) {
      const int q = 2 * k + sd;
      const bool in = sd ? c[k] + 1 < g.n[k] : c[k] > 0;
      nb[q] = in ? (sd ? i + st : i - st) : i;
      const double sn = in ? exp(m[nb[q]]) : si;
      dT[q] = in ? dharm(si, sn) * dm[i] + dharm(sn, si) * dm[nb[q]] : 0.0;
    }
  }
  for (int j = 0; j < ns; ++j) {
    const double* uj = u + size_t(j) * ncell;
    const double ui = uj[i];
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < 6; ++q) acc += dT[q] * (ui - uj[nb[q]]);
    y[size_t(j) * ncell + i] = acc;
  }
}

// Flux weights of the fixed-basis gradient: W_k(i) = -sum_j (u_j(i) - u_j(n))
// (z_j(i) - z_j(n)) for the face between i and n = i + e_k.
__global__ void k_wfixed(GridInfo g, long long ncell, int ns, const double* u, const double* z,
                         double* W) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= ncell) return;
  const int c[3] = {int(i % g.n[0]), int((i / g.n[0]) % g.n[1]), int(i / ((long long)g.n[0] * g.n[1]))};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double acc = 0.0;
    if (c[k] + 1 < g.n[k]) {
      const long long n = i + gstride_of(g, k);
      for (int j = 0; j < ns; ++j) {
        const double* uj = u + size_t(j) * ncell;
        const double* zj = z + size_t(j) * ncell;
        acc -= (uj[i] - uj[n]) * (zj[i] - zj[n]);
      }
    }
    W[k * ncell + i] = acc;
  }
}

// b_j(v) = scale * sum over the column v of S_k of S_k(cell, v) y_j(cell)
// (column lists: cptr over vertices, cidx = S_k entry, ccell = its row).
__global__ void k_restrict(const int* cptr, const int* cidx, const int* ccell, const double* pval,
                           const double* y, int nc, int ns, long long ncell, double scale, double* b) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= (long long)nc * ns) return;
  const int v = int(t % nc), j = int(t / nc);
  const double* yj = y + size_t(j) * ncell;
  double acc = 0.0;
  for (int e = cptr[v]; e < cptr[v + 1]; ++e) acc += pval[cidx[e]] * yj[ccell[e]];
  b[size_t(j) * nc + v] = scale * acc;
}

// rhs_j(i) -= sum_o dK[o](i) t_j(i + off_o) on the coarse grid (27 diagonals)
__global__ void k_coarse_dk_sub(const double* kd, int ldk, int ncx, int ncy, int ncz, int ns,
                                const double* t, double* rhs) {
  const long long tid = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const int nc = ncx * ncy * ncz;
  if (tid >= (long long)nc * ns) return;
  const int i = int(tid % nc), j = int(tid / nc);
  const int x = i % ncx, y = (i / ncx) % ncy, z = i / (ncx * ncy);
  const double* tj = t + size_t(j) * nc;
  double acc = 0.0;
  for (int o = 0; o < 27; ++o) {
    const int dx = o % 3 - 1, dy = (o / 3) % 3 - 1, dz = o / 9 - 1;
    if (x + dx < 0 || x + dx >= ncx || y + dy < 0 || y + dy >= ncy || z + dz < 0 || z + dz >= ncz) continue;
    acc += kd[size_t(o) * ldk + i] * tj[i + dx + ncx * (dy + ncy * dz)];
  }
  rhs[size_t(j) * nc + i] -= acc;
}

__global__ void k_residual(const double* D, const double* dobs, double* v, long long n,
                           double* phi) {
  __shared__ double red[16 * 4];
  double s = 0.0;
  // eight elements a thread per pass, their loads in flight together
  for (long long i0 = threadIdx.x; i0 < n; i0 += 8LL * blockDim.x) {
    double d[8], o[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const long long i = i0 + u * (long long)blockDim.x;
      d[u] = i < n ? D[i] : 0.0;
      o[u] = i < n ? dobs[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const long long i = i0 + u * (long long)blockDim.x;
      if (i >= n) continue;
      const double r = d[u] - o[u];
      v[i] = r;
      s += r * r;
    }
  }
  double arr[1] = {s};
  block_sum<16, 1>(arr, 1, red);
  if (threadIdx.x == 0) phi[0] = 0.5 * arr[0];
}

template <int BLOCK, int CPT, int NCP>
size_t local_lds_bytes(const LocalParams& p, bool adj) {
  const int nw = BLOCK / kWave;
  size_t d = size_t(p.sig_cap) + size_t(NCP) * p.nu_cap + 2 * nw * 40 + (adj ? 128 : 0) + size_t(3) * p.nu_cap;
  return d * sizeof(double);
}

template <int BLOCK, int CPT, int NCP, bool MULTI = false>
hipError_t launch_local_t(const LocalParams& p, bool adj, hipStream_t s) {
  const size_t lds = local_lds_bytes<BLOCK, CPT, NCP>(p, adj);
  if (lds > 160 * 1024) return hipErrorInvalidConfiguration;
  unsigned grid = unsigned(p.nent);
  if constexpr (MULTI) {
    // a fixed grid of as many workgroups as fit the device at once
    const int per_cu = std::max(1, std::min<int>(int((160 * 1024) / std::max<size_t>(lds, 1)), 2048 / BLOCK));
    grid = unsigned(std::min<long long>(p.nent, 256LL * per_cu));
  }
  if (adj) {
    auto kern = k_local_adj<BLOCK, CPT, NCP, MULTI>;
    if (lds > 64 * 1024) (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    hipLaunchKernelGGL(kern, dim3(grid), dim3(BLOCK), lds, s, p);
  } else {
    auto kern = k_local_fwd<BLOCK, CPT, NCP, MULTI>;
    if (lds > 64 * 1024) (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    hipLaunchKernelGGL(kern, dim3(grid), dim3(BLOCK), lds, s, p);
  }
  return hipGetLastError();
}

// The generic variants, by own-cell count (and corners): index i of
// kClassLocalFirst + i.
int generic_index(const LocalParams& p) {
  const int nu = p.nu_cap;
  if (nu <= 64) return 0;
  if (nu <= 128) return 1;
  if (nu <= 256) return p.nc_cap <= 4 ? 2 : 3;  // faces (4 corners): all corners in one pass
  if (nu <= 384) return 4;
  if (nu <= 512) return 5;
  if (nu <= 1024) return 6;
  // LDS: sigma, one direction, tp (four cells a thread at 1024 threads spilled
  // more and ran 1.7x slower at r = 16)
  if (nu <= 4096) return 7;
  return -1;
}

template <bool MULTI>
hipError_t launch_generic(int idx, const LocalParams& p, bool adj, hipStream_t s) {
  switch (idx) {
    case 0: return launch_local_t<64, 1, 8, MULTI>(p, adj, s);
    case 1: return launch_local_t<128, 1, 8, MULTI>(p, adj, s);
    case 2: return launch_local_t<256, 1, 4, MULTI>(p, adj, s);
    case 3: return launch_local_t<256, 1, 8, MULTI>(p, adj, s);
    case 4: return launch_local_t<384, 1, 8, MULTI>(p, adj, s);
    case 5: return launch_local_t<512, 1, 8, MULTI>(p, adj, s);
    case 6: return launch_local_t<1024, 1, 4, MULTI>(p, adj, s);
    case 7: return launch_local_t<512, 8, 1, MULTI>(p, adj, s);
    default: return hipErrorInvalidConfiguration;
  }
}

hipError_t launch_local(const LocalParams& p, bool adj, hipStream_t s) {
  if (p.nent == 0) return hipSuccess;
  if (wave_path_fits(p)) return launch_wave_local(p, adj, s);
  return launch_generic<false>(generic_index(p), p, adj, s);
}

}  // namespace

template <int BLOCK, int CPT, int NCP>
hipError_t launch_tan_generic_t(const LocalParams& p, hipStream_t s) {
  const size_t lds = local_lds_bytes<BLOCK, CPT, NCP>(p, false);
  if (lds > 160 * 1024) return hipErrorInvalidConfiguration;
  auto kern = k_local_tan<BLOCK, CPT, NCP>;
  if (lds > 64 * 1024) (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  hipLaunchKernelGGL(kern, dim3(p.nent), dim3(BLOCK), lds, s, p);
  return hipGetLastError();
}

hipError_t launch_local_tan(const LocalParams& p, hipStream_t s) {
  if (p.nent == 0) return hipSuccess;
  if (!p.dm || !p.dpval) return hipErrorInvalidValue;
  if (wave_path_fits(p)) return launch_wave_tan(p, s);
  switch (generic_index(p)) {
    case 0: return launch_tan_generic_t<64, 1, 8>(p, s);
    case 1: return launch_tan_generic_t<128, 1, 8>(p, s);
    case 2: return launch_tan_generic_t<256, 1, 4>(p, s);
    case 3: return launch_tan_generic_t<256, 1, 8>(p, s);
    case 4: return launch_tan_generic_t<384, 1, 8>(p, s);
    case 5: return launch_tan_generic_t<512, 1, 8>(p, s);
    case 6: return launch_tan_generic_t<1024, 1, 4>(p, s);
    case 7: return launch_tan_generic_t<512, 8, 1>(p, s);
    default: return hipErrorInvalidConfiguration;
  }
}

int local_class(const LocalParams& p) {
  if (wave_path_fits(p)) return wave_class(p);
  const int idx = generic_index(p);
  return idx < 0 ? kClassNone : kClassLocalFirst + idx;
}

int full_class(int u) { return u == 7 ? kClassFull7 : (u == 3 ? kClassFull3 : kClassNone); }

int faces_class(int u) { return u == 7 ? kClassFaces7 : (u == 3 ? kClassFaces3 : kClassNone); }

int local_class_uni_cap(const LocalParams& p, int klass) {
  return klass < kClassLocalFirst ? wave_class_uni_cap(p, klass) : 0;
}

hipError_t launch_local_multi(const LocalParams& p, int klass, bool adj, hipStream_t s) {
  if (p.nent == 0) return hipSuccess;
  if (!p.multi || !p.items) return hipErrorInvalidValue;
  if (klass >= kClassLocalFirst) return launch_generic<true>(klass - kClassLocalFirst, p, adj, s);
  return launch_wave_multi(p, klass, adj, s);
}

hipError_t launch_edge_multi(const LocalParams& p, bool adj, hipStream_t s) {
  if (p.nent == 0) return hipSuccess;
  if (!p.multi || !p.items) return hipErrorInvalidValue;
  if (p.line_cap <= 0 || p.line_cap > kMaxLine) return hipErrorInvalidConfiguration;
  if (p.line_cap <= 9)
    hipLaunchKernelGGL(k_edge_multi<9>, dim3((p.nent + 127) / 128), dim3(128), 0, s, p, adj ? 1 : 0);
  else
    hipLaunchKernelGGL(k_edge_multi<kMaxLine>, dim3((p.nent + 127) / 128), dim3(128), 0, s, p, adj ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_check_finite(const double* m, long long n, int* status, hipStream_t s) {
  const int threads = 256;
  long long blocks = (n + threads - 1) / threads;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_check_finite, dim3(unsigned(blocks)), dim3(threads), 0, s, m, n, status);
  return hipGetLastError();
}

hipError_t launch_edge_fwd(const LocalParams& p, int lagrange, hipStream_t s) {
  if (p.nent == 0) return hipSuccess;
  if (p.line_cap <= 0 || p.line_cap > kMaxLine) return hipErrorInvalidConfiguration;
  if (p.line_cap <= 9)
    hipLaunchKernelGGL(k_edge_fwd<9>, dim3((p.nent + 63) / 64), dim3(64), 0, s, p, lagrange);
  else
    hipLaunchKernelGGL(k_edge_fwd<kMaxLine>, dim3((p.nent + 63) / 64), dim3(64), 0, s, p, lagrange);
  return hipGetLastError();
}

hipError_t launch_edge_adj(const LocalParams& p, int lagrange, hipStream_t s) {
  if (p.nent == 0) return hipSuccess;
  if (p.line_cap <= 0 || p.line_cap > kMaxLine) return hipErrorInvalidConfiguration;
  if (p.line_cap <= 9)
    hipLaunchKernelGGL(k_edge_adj<9>, dim3((p.nent + 63) / 64), dim3(64), 0, s, p, lagrange);
  else
    hipLaunchKernelGGL(k_edge_adj<kMaxLine>, dim3((p.nent + 63) / 64), dim3(64), 0, s, p, lagrange);
  return hipGetLastError();
}

hipError_t launch_local_fwd(const LocalParams& p, int, hipStream_t s) { return launch_local(p, false, s); }
hipError_t launch_local_adj(const LocalParams& p, int, hipStream_t s) { return launch_local(p, true, s); }

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
  const long long n = (long long)(bytes / 4);
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_words, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s,
                     static_cast<unsigned*>(p), n);
  return hipGetLastError();
}

hipError_t launch_copy(double* dst, const double* src, long long n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_d, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, dst, src, n);
  return hipGetLastError();
}

hipError_t launch_set_ones(const int* idx, int n, double* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_set_ones, dim3((n + 255) / 256), dim3(256), 0, s, idx, n, out);
  return hipGetLastError();
}

hipError_t launch_kassemble(const int* kcptr, const int* kcidx, const int* dslot, const double* kent,
                            double* kval, double* kdia, int nnz, hipStream_t s) {
  if (nnz == 0) return hipSuccess;
  hipLaunchKernelGGL(k_kassemble, dim3((nnz + 255) / 256), dim3(256), 0, s, kcptr, kcidx, dslot, kent,
                     kval, kdia, nnz);
  return hipGetLastError();
}

hipError_t launch_gather_slots(const int* slot_dst, const int* slot_ptr, const int* ent_pidx,
                               const double* ent_w, const int* ent_col, const double* colw,
                               int colw_ld, const double* pval, double* out, int nslot, int ncol,
                               int nc, hipStream_t s) {
  const long long n = (long long)nslot * ncol;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_slots, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, slot_dst,
                     slot_ptr, ent_pidx, ent_w, ent_col, colw, colw_ld, pval, out, nslot, ncol, nc);
  return hipGetLastError();
}

hipError_t launch_data(const int* rptr, const int* rcell, const double* rval, int nr, int ns,
                       const int* prow, const int* pcol, const double* pval, const double* t,
                       int nc, double* D, hipStream_t s, int accumulate) {
  const int n = nr * ns;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_data, dim3((n + 255) / 256), dim3(256), 0, s, rptr, rcell, rval, nr, ns, prow,
                     pcol, pval, t, nc, D, accumulate);
  return hipGetLastError();
}

int prolong_ldt(int ns) { return (std::max(ns, 1) + 3) / 4 * 4; }

hipError_t launch_prolong(const int* prow, const int* pcol, const double* pval, const double* t,
                          const int ncv[3], int ns, long long ncell, double* u, double* scratch, hipStream_t s) {
  const int ldt = prolong_ldt(ns);
  const int nc = ncv[0] * ncv[1] * ncv[2];
  const long long nt = (long long)nc * ldt;
  hipLaunchKernelGGL(k_transpose_t, dim3(unsigned((nt + 255) / 256)), dim3(256), 0, s, t, nc, ns, ldt, scratch);
  // the LDS box of vertex rows, where it fits in 64 KB
  const size_t box = size_t(kProlongK) * kProlongJ * ncv[0] * (ldt + 2) * sizeof(double);
  const int staged = box <= 64 * 1024 ? 1 : 0;
  hipLaunchKernelGGL(k_prolong, dim3(unsigned((ncell + 255) / 256)), dim3(256), staged ? box : 0, s, prow, pcol,
                     pval, scratch, ldt, ns, ncv[0], ncv[1], nc, ncell, staged, u);
  return hipGetLastError();
}

hipError_t launch_sload(int nelec, const int* ecell, const int* rptr, const int* ridx,
                        const double* rw, const int* sptr, const int* sidx, const double* sw,
                        const int* prow, const int* pcol, const double* t, const double* lam,
                        const double* v, int nc, int ns, int nr, double* sload, hipStream_t s) {
  if (nelec == 0) return hipSuccess;
  const int n = nelec * 8;
  hipLaunchKernelGGL(k_sload, dim3((n + 255) / 256), dim3(256), 0, s, nelec, ecell, rptr, ridx, rw,
                     sptr, sidx, sw, prow, pcol, t, lam, v, nc, ns, nr, sload);
  return hipGetLastError();
}

hipError_t launch_gfinal(const double* sig, const double* W, GridInfo g, long long ncell, double* grad,
                         hipStream_t s) {
  if (ncell <= 0) return hipSuccess;
  if (ncell >= (1LL << 31)) return hipErrorInvalidValue;
  const int spans = int((ncell + 255) / 256);
  const int spx = (spans + 7) / 8;
  hipLaunchKernelGGL(k_gfinal, dim3(8u * unsigned(spx)), dim3(256), 0, s, sig, W, g, int(ncell), spx, grad);
  return hipGetLastError();
}

hipError_t launch_prep_model(double* dst, double* sig, const double* src, long long n, int* status,
                             hipStream_t s) {
  const long long blocks = std::min<long long>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_prep_model, dim3(unsigned(std::max<long long>(blocks, 1))), dim3(256), 0, s, dst, sig,
                     src, n, status);
  return hipGetLastError();
}

hipError_t launch_edge_tan(const LocalParams& p, int lagrange, hipStream_t s) {
  if (p.nent == 0) return hipSuccess;
  hipLaunchKernelGGL(k_edge_tan, dim3((p.nent + 63) / 64), dim3(64), 0, s, p, lagrange);
  return hipGetLastError();
}

hipError_t launch_dAu(const double* m, const double* dm, GridInfo g, long long ncell, int ns,
                      const double* u, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_dAu, dim3(unsigned((ncell + 255) / 256)), dim3(256), 0, s, m, dm, g, ncell, ns, u, y);
  return hipGetLastError();
}

hipError_t launch_wfixed(GridInfo g, long long ncell, int ns, const double* u, const double* z, double* W,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_wfixed, dim3(unsigned((ncell + 255) / 256)), dim3(256), 0, s, g, ncell, ns, u, z, W);
  return hipGetLastError();
}

hipError_t launch_restrict(const int* cptr, const int* cidx, const int* ccell, const double* pval,
                           const double* y, int nc, int ns, long long ncell, double scale, double* b,
                           hipStream_t s) {
  const long long n = (long long)nc * ns;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_restrict, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, cptr, cidx, ccell, pval, y,
                     nc, ns, ncell, scale, b);
  return hipGetLastError();
}

hipError_t launch_coarse_dk_sub(const double* kd, int ldk, const int ncv[3], int ns, const double* t,
                                double* rhs, hipStream_t s) {
  const long long n = (long long)ncv[0] * ncv[1] * ncv[2] * ns;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_coarse_dk_sub, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, kd, ldk, ncv[0], ncv[1],
                     ncv[2], ns, t, rhs);
  return hipGetLastError();
}

hipError_t launch_residual(const double* D, const double* dobs, double* v, long long n, double* phi,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_residual, dim3(1), dim3(1024), 0, s, D, dobs, v, n, phi);
  return hipGetLastError();
}

}  // namespace msfv
