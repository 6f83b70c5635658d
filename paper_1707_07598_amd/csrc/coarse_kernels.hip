// Coarse solves of the pinned Galerkin system A_k t = S_k^T q (Sec. 3,
// reduced forward problem) and of its transpose for the adjoint (Sec. 4.3).
//
// A_k is a 27-point stencil on the coarse-vertex grid, stored as 27 padded
// diagonals.  One workgroup solves one right-hand side with preconditioned
// CG: the search direction lives in LDS with a zero halo, so the stencil
// loop is branch-free and every thread issues its coefficient loads back to
// back.  Vertex 0 is fixed (t_0 = 0): its row and column drop out.
//
// Preconditioners:
//  * Jacobi, M^-1 = D^-1;
//  * two-level additive, M^-1 = D^-1 + Z E^-1 Z^T, with Z the indicator
//    columns of boxes ("aggregates") of coarse vertices and E = Z^T A_k Z.
//    E^-1 (at most 64 x 64) is formed once per operator by a setup kernel and
//    kept in LDS by the solver.  On heterogeneous media this removes the
//    slowest error components of the Jacobi iteration and cuts the
//    iteration count by a factor of two or more.
// All reductions (dot products, aggregate sums) run in a fixed order, so
// results are bit-reproducible.
#include "kernels.hpp"

namespace msfv {

namespace {

constexpr int kWave = 64;

// DPP lane exchange of a double within 16-lane rows (every lane written).
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}

// Sum over each 16-lane row (quad pairs, quads, half rows, rows); every lane
// of the row ends with the same bits, since each step adds two equal-order
// partials in either order.
__device__ __forceinline__ double row16_sum(double v) {
  v += dpp_move<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_move<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_move<0x141>(v);  // row_half_mirror
  v += dpp_move<0x140>(v);  // row_mirror
  return v;
}

// v[l] + v[l ^ 16] (ROW32 = false) or v[l] + v[l ^ 32] (ROW32 = true) in every
// lane, from the gfx950 row-swap instructions applied to two copies of v.
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

// Wavefront sum, bitwise identical in every lane.
__device__ __forceinline__ double wsum(double v) {
  return swap_add<true>(swap_add<false>(row16_sum(v)));
}

// Sum NV values over the workgroup; every thread receives the totals (waves
// added in a fixed order).  red holds NW * NV doubles and must not be reused
// by the next call before every thread has read it (alternate two buffers).
template <int NW, int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* red) {
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wsum(v[i]);
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) red[wid * NV + i] = v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double s = red[i];
    // four partials in flight at a time: with all of them loaded at once the
    // 1024-thread PCG kernel spills (132 bytes of scratch at 4 rows a thread)
#pragma unroll 4
    for (int w = 1; w < NW; ++w) s += red[w * NV + i];
    v[i] = s;
  }
}

__device__ __forceinline__ int agg_index(const CoarseDefl& d, int x, int y, int z) {
  return x / d.b[0] + d.na3[0] * (y / d.b[1] + d.na3[1] * (z / d.b[2]));
}

// out[a] = sum of stage over the vertices of aggregate a, 16 lanes per
// aggregate, each lane striding over the aggregate's vertex list in a fixed
// order.  aoff: the list offsets of the na aggregates (na + 1); apos: the
// position in stage of each listed vertex (both in LDS).
template <int BLOCK>
__device__ __forceinline__ void aggregate_sums(const double* stage, int na, const int* aoff, const int* apos,
                                               double* out) {
  const int grp = threadIdx.x >> 4, l = threadIdx.x & 15;
  for (int a = grp; a < na; a += BLOCK / 16) {
    const int k0 = aoff[a], k1 = aoff[a + 1];
    double s = 0.0;
    for (int k = k0 + l; k < k1; k += 16) s += stage[apos[k]];
    s = row16_sum(s);
    if (l == 0) out[a] = s;
  }
}

// ---------------------------------------------------------------------------
// E = Z^T A_k Z over the free vertices (vertex 0 excluded), one wave per
// aggregate a: each lane walks its share of the box's vertices and adds
// every stencil coefficient K_ij into one of 27 accumulators, by the
// direction D from a to the aggregate of j (each axis steps out of the box
// only from the box face on that side); the wave sums are E[a][a + D], and
// the wave writes row a of E (zeros elsewhere) to the global buffer e.
__global__ __launch_bounds__(kWave) void k_coarse_defl_assemble(const double* __restrict__ kdia, int ldk,
                                                                int ncx, int ncy, int ncz, CoarseDefl d,
                                                                double* e) {
  const int na = d.na;
  const int a = blockIdx.x, l = threadIdx.x;
  const int ax = a % d.na3[0], ay = (a / d.na3[0]) % d.na3[1], az = a / (d.na3[0] * d.na3[1]);
  const int x0 = ax * d.b[0], y0 = ay * d.b[1], z0 = az * d.b[2];
  const int w = min(d.b[0], ncx - x0), h = min(d.b[1], ncy - y0), dd = min(d.b[2], ncz - z0);
  const int cnt = w * h * dd;
  double acc[27];
#pragma unroll
  for (int D = 0; D < 27; ++D) acc[D] = 0.0;
  for (int k = l; k < cnt; k += kWave) {
    const int x = x0 + k % w, y = y0 + (k / w) % h, z = z0 + k / (w * h);
    const int i = x + ncx * (y + ncy * z);
    if (i == 0) continue;
    const bool lo[3] = {x == x0, y == y0, z == z0};
    const bool hi[3] = {x == x0 + w - 1, y == y0 + h - 1, z == z0 + dd - 1};
#pragma unroll
    for (int o = 0; o < 27; ++o) {
      const int ox = o % 3 - 1, oy = (o / 3) % 3 - 1, oz = o / 9 - 1;
      if (i + ox + ncx * (oy + ncy * oz) == 0) continue;  // the fixed vertex
      const double v = kdia[size_t(o) * ldk + i];
      // aggregate step on each axis
      const int sx = ox < 0 ? (lo[0] ? -1 : 0) : (ox > 0 ? (hi[0] ? 1 : 0) : 0);
      const int sy = oy < 0 ? (lo[1] ? -1 : 0) : (oy > 0 ? (hi[1] ? 1 : 0) : 0);
      const int sz = oz < 0 ? (lo[2] ? -1 : 0) : (oz > 0 ? (hi[2] ? 1 : 0) : 0);
      // candidate directions of this offset: 0 or the offset's own step per axis
#pragma unroll
      for (int cz = 0; cz < (oz ? 2 : 1); ++cz)
#pragma unroll
        for (int cy = 0; cy < (oy ? 2 : 1); ++cy)
#pragma unroll
          for (int cx = 0; cx < (ox ? 2 : 1); ++cx) {
            const int Dx = cx ? ox : 0, Dy = cy ? oy : 0, Dz = cz ? oz : 0;
            const bool hit = sx == Dx && sy == Dy && sz == Dz;
            acc[(Dx + 1) + 3 * (Dy + 1) + 9 * (Dz + 1)] += hit ? v : 0.0;
          }
    }
  }
#pragma unroll
  for (int D = 0; D < 27; ++D) acc[D] = wsum(acc[D]);
  // row a: lane b writes E[a][b] (and b + 64 ... for larger na)
  for (int b = l; b < na; b += kWave) {
    const int bx = b % d.na3[0], by = (b / d.na3[0]) % d.na3[1], bz = b / (d.na3[0] * d.na3[1]);
    const int Dx = bx - ax, Dy = by - ay, Dz = bz - az;
    double v = 0.0;
#pragma unroll
    for (int D = 0; D < 27; ++D)
      if (Dx == D % 3 - 1 && Dy == (D / 3) % 3 - 1 && Dz == D / 9 - 1) v = acc[D];
    e[size_t(a) * na + b] = v;
  }
}

// The inverse of E (read from e, which may alias einv), by one workgroup:
// Gauss-Jordan (E is SPD, so no pivoting), lane = column, 16 waves sharing
// the rows, one barrier a step; the symmetric part is written to einv.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_coarse_defl_setup(const double* e, CoarseDefl d,
                                                             double* einv, int* status) {
  extern __shared__ double lds[];
  const int na = d.na;
  // two copies of E (row-major): step k reads one and writes the other, so a
  // step needs one barrier
  double* cur = lds;
  double* nxt = lds + na * na;
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  for (int i = threadIdx.x; i < na * na; i += BLOCK) cur[i] = e[i];
  __syncthreads();
  const int j = threadIdx.x % kWave, rg = threadIdx.x / kWave;
  constexpr int NRG = BLOCK / kWave;
  for (int k = 0; k < na; ++k) {
    const double piv = cur[k * na + k];
    const double inv = 1.0 / piv;
    const double rk = j < na ? (j == k ? inv : cur[k * na + j] * inv) : 0.0;
    if (threadIdx.x == 0 && !(piv > 0.0)) bad = 1;
    if (j < na) {
#pragma unroll
      for (int t = 0; t < 64 / NRG; ++t) {
        const int i = rg + t * NRG;
        if (i >= na) continue;
        const double f = cur[i * na + k];
        if (i == k)
          nxt[i * na + j] = rk;
        else
          nxt[i * na + j] = j == k ? -f * inv : cur[i * na + j] - f * rk;
      }
    }
    __syncthreads();
    double* t = cur;
    cur = nxt;
    nxt = t;
  }
  double* E = cur;
  if (threadIdx.x == 0 && bad) atomicAdd(status + kStCoarseNoconv, 1);
  // symmetric part (the exact inverse is symmetric)
  for (int t = threadIdx.x; t < na * na; t += BLOCK) {
    const int r = t / na, c = t % na;
    einv[t] = 0.5 * (E[r * na + c] + E[c * na + r]);
  }
}

// ---------------------------------------------------------------------------
// PCG on the 27-diagonal operator, one workgroup per column.  Rows are padded
// to ldk = RPT*BLOCK (padding rows have zero diagonals); the search direction
// p lives in LDS with a zero halo, so the stencil loop has no branches.
// Row layouts (QM):
//  * 0: thread t owns rows t + q*BLOCK; p in LDS by row;
//  * 1 and 2 (RPT = 2, 4, 6): thread t owns the RPT consecutive rows RPT*t + q, so
//    it loads its coefficients of one offset as RPT contiguous doubles and
//    shares the x-neighbours of its rows; p in LDS as RPT planes, row j (after
//    a halo shift) in plane j mod RPT, slot j div RPT (consecutive lanes,
//    consecutive slots).  The window of a (dy, dz) row shift o starts at
//    plane o mod RPT, so Ncx need not be a multiple of RPT (layout 2; layout
//    1 is the same with the plane offsets fixed at compile time, for
//    RPT | Ncx).
// With DEFL, the LDS copy of p is reused between the stencil product and the
// update of p to stage r for the aggregate sums.
template <int BLOCK, int RPT, bool DEFL, int QM>
__global__ __launch_bounds__(BLOCK) void k_coarse_pcg(const double* __restrict__ kdia, int ldk, int ncx,
                                                      int ncy, int ncz, const double* __restrict__ rhs,
                                                      double* __restrict__ xout, double rtol, int maxit,
                                                      CoarseDefl d, int* status,
                                                      unsigned long long* work) {
  extern __shared__ double lds[];
  constexpr int NW = BLOCK / kWave;
  const int nc = ncx * ncy * ncz;
  const int pad = 1 + ncx + (ncz > 1 ? ncx * ncy : 0);  // a 2-D grid has no z-neighbours
  const int H = pad / RPT + 2;              // QM: halo slots a plane side
  const int plane = BLOCK + 2 * H;          // QM: slots a plane
  const int pn = QM != 0 ? RPT * plane : ldk + 2 * pad;
  double* p = QM != 0 ? lds : lds + pad;
  // LDS position of row i (any row within the halo)
  auto pos = [=](int i) -> int {
    if (QM == 0) return i;
    const int jj = i + RPT * H;
    return (jj % RPT) * plane + jj / RPT;
  };
  auto row = [=](int q) -> int { return QM != 0 ? RPT * int(threadIdx.x) + q : int(threadIdx.x) + q * BLOCK; };
  double* redA = lds + pn;
  double* redB = redA + NW * 4;
  double* einv = redB + NW * 4;        // DEFL: na * na
  double* sv = einv + (DEFL ? d.na * d.na : 0);  // DEFL: 64
  double* yv = sv + 64;                // DEFL: 64
  // DEFL: the aggregates' vertex-list offsets (na + 1 <= 65) and the LDS
  // position of every listed vertex, read from the table once
  int* aoff = reinterpret_cast<int*>(yv + 64);
  int* apos = aoff + 72;
  for (int i = threadIdx.x; i < pn; i += BLOCK) lds[i] = 0.0;
  if (DEFL) {
    for (int i = threadIdx.x; i < d.na * d.na; i += BLOCK) einv[i] = d.einv[i];
    for (int a = threadIdx.x; a <= d.na; a += BLOCK) aoff[a] = d.arows[a];
    for (int k = threadIdx.x; k < nc; k += BLOCK) apos[k] = pos(d.arows[d.na + 1 + k]);
  }
  __syncthreads();
  const double* b = rhs + size_t(blockIdx.x) * nc;
  double* xo = xout + size_t(blockIdx.x) * nc;
  // with many rows a thread the iterate x lives in the output buffer instead
  // of registers (the per-thread state otherwise spills)
  constexpr bool LEAN = RPT > 4;
  double x[LEAN ? 1 : RPT], r[RPT], pv[RPT], dinv[RPT];
  unsigned agg[(RPT + 3) / 4];  // DEFL: aggregate of row q in byte q % 4 of agg[q / 4]
#pragma unroll
  for (int q = 0; q < (RPT + 3) / 4; ++q) agg[q] = 0u;
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int i = row(q);
    if (!LEAN) x[q] = 0.0;
    if (LEAN && i < nc) xo[i] = 0.0;
    r[q] = pv[q] = dinv[q] = 0.0;
    if (i >= nc || i == 0) continue;  // vertex 0 is fixed: its row and column drop out
    const double dg = kdia[13 * ldk + i];
    dinv[q] = dg > 0.0 ? 1.0 / dg : 0.0;
    r[q] = b[i];
    if (DEFL)
      agg[q / 4] |= unsigned(agg_index(d, i % ncx, (i / ncx) % ncy, i / (ncx * ncy))) << (8 * (q % 4));
  }

  // Aggregate correction y = E^-1 Z^T r into yv (r staged in the LDS copy of
  // p, which is free between the stencil product and the update of p).
  auto coarse_correction = [&]() {
#pragma unroll
    for (int q = 0; q < RPT; ++q) p[pos(row(q))] = r[q];
    __syncthreads();
    aggregate_sums<BLOCK>(p, d.na, aoff, apos, sv);
    __syncthreads();
    // y = E^-1 s: 16 lanes per row of E^-1 (symmetric, read along a row),
    // each lane a strided share of the columns, then the row sum
    for (int t = int(threadIdx.x) >> 4; t < d.na; t += BLOCK / 16) {
      const int l = threadIdx.x & 15;
      double y = 0.0;
      for (int c = l; c < d.na; c += 16) y += einv[t * d.na + c] * sv[c];
      y = row16_sum(y);
      if (l == 0) yv[t] = y;
    }
    __syncthreads();
  };
  // z = M^-1 r for row q (DEFL: after coarse_correction)
  auto zrow = [&](int q) -> double {
    double z = r[q] * dinv[q];
    if (DEFL && dinv[q] != 0.0) z += yv[(agg[q / 4] >> (8 * (q % 4))) & 0xFFu];
    return z;
  };

  if (DEFL) coarse_correction();
  double s0[2] = {0.0, 0.0};
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    pv[q] = zrow(q);
    s0[0] += r[q] * r[q];
    s0[1] += r[q] * pv[q];
  }
  block_sum<NW, 2>(s0, redA);  // its barrier also orders the staging reads before the writes below
  const double bb = s0[0];
  double rz = s0[1];
  // r.r of the current iterate, kept in scalar registers (the value is the
  // same in every lane)
  auto uniform = [](double v) {
    const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
    const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
    return __hiloint2double(hi, lo);
  };
  double last = uniform(bb);
  bool done = !(bb > 0.0);
  const double tol2 = rtol * rtol;
  const bool owns_pin = threadIdx.x == 0;
#pragma unroll
  for (int q = 0; q < RPT; ++q) p[pos(row(q))] = pv[q];
  __syncthreads();
  int it = 0;
  bool ok = true;
  while (!done) {
    if (it >= maxit) {
      ok = false;
      break;
    }
    ++it;
    double ap[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) ap[q] = 0.0;
    // Opaque copies of the uniform base and the lane offset: the 27*RPT
    // coefficient addresses are formed here (scalar base + one lane offset)
    // instead of being hoisted out of the loop and spilled.
    const double* kb = kdia;
    int lo = threadIdx.x;
    asm volatile("" : "+s"(kb));
    asm volatile("" : "+v"(lo));
    if (QM == 0) {
#pragma unroll
      for (int dz = -1; dz <= 1; ++dz) {
        if (dz != 0 && ncz == 1) continue;  // 2-D: no z-neighbours (and no z-halo)
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
          for (int dx = -1; dx <= 1; ++dx) {
            const int o = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
            const int off = dx + ncx * (dy + ncy * dz);
            const double* kd = kb + size_t(o) * ldk;
#pragma unroll
            for (int q = 0; q < RPT; ++q) ap[q] += kd[q * BLOCK + lo] * p[lo + q * BLOCK + off];
          }
      }
    } else {
#pragma unroll
      for (int dz = -1; dz <= 1; ++dz) {
        if (dz != 0 && ncz == 1) continue;  // 2-D: no z-neighbours (and no z-halo)
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy) {
          // window w[s] = p(row RPT*t + o + s), s = -1 .. RPT, for the row
          // shift o = Ncx (dy + Ncy dz) = RPT m + c, 0 <= c < RPT: row
          // RPT (t + m) + (c + s) sits in plane (c + s) mod RPT, slot
          // t + m + floor((c + s) / RPT)
          double wv[RPT + 2];
          if (QM == 1) {  // RPT | Ncx: c = 0
            const int slot = lo + H + (ncx * (dy + ncy * dz)) / RPT;
            wv[0] = p[(RPT - 1) * plane + slot - 1];
#pragma unroll
            for (int q = 0; q < RPT; ++q) wv[q + 1] = p[q * plane + slot];
            wv[RPT + 1] = p[slot + 1];
          } else {
            const int oyz = ncx * (dy + ncy * dz);
            const int m = oyz >= 0 ? oyz / RPT : -((RPT - 1 - oyz) / RPT);
            const int c = oyz - m * RPT;
            const int slot = lo + H + m;
#pragma unroll
            for (int s = -1; s <= RPT; ++s) {
              const int e = c + s + RPT;  // in [RPT - 1, 3 RPT)
              wv[s + 1] = p[(e % RPT) * plane + slot + e / RPT - 1];
            }
          }
#pragma unroll
          for (int dx = -1; dx <= 1; ++dx) {
            const int o = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
            const double2* kd = reinterpret_cast<const double2*>(kb + size_t(o) * ldk) + lo * (RPT / 2);
#pragma unroll
            for (int h = 0; h < RPT / 2; ++h) {
              const double2 kv = kd[h];
              ap[2 * h] += kv.x * wv[2 * h + 1 + dx];
              ap[2 * h + 1] += kv.y * wv[2 * h + 2 + dx];
            }
          }
        }
      }
    }
    if (owns_pin) ap[0] = 0.0;
    double pq[1] = {0.0};
#pragma unroll
    for (int q = 0; q < RPT; ++q) pq[0] += pv[q] * ap[q];
    block_sum<NW, 1>(pq, redA);  // also: every thread is past its stencil reads of p
    const double alpha = pq[0] != 0.0 ? rz / pq[0] : 0.0;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      if (!LEAN) {
        x[q] += alpha * pv[q];
      } else {
        const int i = row(q);
        if (i < nc) xo[i] += alpha * pv[q];
      }
      r[q] -= alpha * ap[q];
    }
    double s2[2] = {0.0, 0.0};
    if constexpr (DEFL) {
      // r.z = r.D^-1 r + y.s with s = Z^T r and y = E^-1 s, so the sums of
      // r.r and r.D^-1 r share the barriers of the aggregate correction:
      // r staged in the LDS copy of p (every thread is past its stencil
      // reads) together with their wave sums ...
      const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        p[pos(row(q))] = r[q];
        s2[0] += r[q] * r[q];
        s2[1] += r[q] * (r[q] * dinv[q]);
      }
      s2[0] = wsum(s2[0]);
      s2[1] = wsum(s2[1]);
      if (lane == 0) {
        redB[2 * wid] = s2[0];
        redB[2 * wid + 1] = s2[1];
      }
      __syncthreads();
      // ... s and the workgroup sums ...
      aggregate_sums<BLOCK>(p, d.na, aoff, apos, sv);
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        double t = redB[i];
#pragma unroll 4  // (see block_sum)
        for (int w = 1; w < NW; ++w) t += redB[2 * w + i];
        s2[i] = t;
      }
      __syncthreads();
      // ... y, and the wave sums of y_t s_t (redA: its p.Ap sums were read
      // before the first barrier above)
      double ys = 0.0;
      for (int t = int(threadIdx.x) >> 4; t < d.na; t += BLOCK / 16) {
        const int l = threadIdx.x & 15;
        double y = 0.0;
        for (int c = l; c < d.na; c += 16) y += einv[t * d.na + c] * sv[c];
        y = row16_sum(y);
        if (l == 0) {
          yv[t] = y;
          ys += y * sv[t];
        }
      }
      ys = wsum(ys);
      if (lane == 0) redA[wid] = ys;
      __syncthreads();
      double yst = redA[0];
#pragma unroll 4  // (see block_sum)
      for (int w = 1; w < NW; ++w) yst += redA[w];
      s2[1] += yst;
    } else {
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        s2[0] += r[q] * r[q];
        s2[1] += r[q] * zrow(q);
      }
      block_sum<NW, 2>(s2, redB);
    }
    last = uniform(s2[0]);
    if (s2[0] <= tol2 * bb) break;
    if (s2[0] != s2[0]) {
      ok = false;
      break;
    }
    const double beta = rz != 0.0 ? s2[1] / rz : 0.0;
    rz = s2[1];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      pv[q] = zrow(q) + beta * pv[q];
      p[pos(row(q))] = pv[q];
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int i = row(q);
    if (!LEAN && i < nc) xo[i] = x[q];
  }
  if (threadIdx.x == 0) {
    atomicMax(status + kStCoarseMaxIt, it);
    if (!ok) atomicAdd(status + kStCoarseNoconv, 1);
    if (bb > 0.0) note_residual(status, kStCoarseRes, last / bb);
    if (work) atomicAdd(work, (unsigned long long)it * (unsigned long long)nc);
  }
}


// ---------------------------------------------------------------------------
// Large coarse systems (more rows than one workgroup can stage in LDS):
// Jacobi-PCG for all right-hand sides together, one launch per phase:
//   spmv_dot : q_j = A p_j and per-tile partials of p_j.q_j (the coefficients
//              of a tile of rows are loaded once for a group of kMG sources);
//   update   : alpha_j from the partials, x_j += alpha p_j, r_j -= alpha q_j,
//              partials of r_j.z_j and r_j.r_j (z = D^-1 r);
//   pupdate  : beta_j and the stop test from the partials, p_j = z_j + beta p_j.
// Every workgroup sums the per-tile partials itself, in tile order, so all
// agree bit for bit without a separate scalar launch.  Per-source scalars
// that a phase both reads and writes are double-buffered by iteration parity.
constexpr int kMT = 256;  // rows per tile (one per thread)
constexpr int kMG = 4;    // sources per stencil workgroup (8: 39 us, 4: 28 us, 2: 33 us, 1: 37 us at 36^3, 27 sources)

// The per-row kernels run on a 1-D grid whose workgroups go round-robin over
// the eight XCDs (linear id mod 8).  Linear id L maps to (tile, column) so
// that XCD x takes the contiguous tiles [x*tpx, (x+1)*tpx) of every column:
// a tile's rows, their stencil halo and their coefficients then stay in one
// XCD's L2 across the columns.  Returns false for the ids past the last tile.
__device__ __forceinline__ bool xcd_tile(int ntile, int& tile, int& col) {
  const int tpx = (ntile + 7) / 8, L = blockIdx.x;
  const int x = L % 8, k = L / 8;
  tile = x * tpx + k % tpx;
  col = k / tpx;
  return tile < ntile;
}
inline unsigned xcd_grid(int ntile, int ncol) { return 8u * unsigned((ntile + 7) / 8) * unsigned(ncol); }

struct CgmState {
  double* r;      // ns * nc
  double* p;      // ns * nc
  double* q;      // ns * nc
  double* part;   // 3 * ns * ntile: p.q, r.D^-1 r, r.r
  double* scal;   // per source: rz[2], bb
  double* s;      // two-level: per source 64 aggregate sums Z^T r
  double* y;      // two-level: per source E^-1 s (64)
  double* sy;     // two-level: per source s.y
  int* flag;      // per source: done[2], unused
};

template <int NW>
__device__ __forceinline__ double tile_sum(double v, double* red) {
  v = wsum(v);
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double t = red[0];
  for (int w = 1; w < NW; ++w) t += red[w];
  return t;
}

// Sum of ntile per-tile partials by wave 0 (lane l adds tiles l, l+64, ...,
// then a fixed-order wave sum), broadcast through LDS; call from every thread.
__device__ __forceinline__ double sum_parts(const double* part, int ntile, double* slot) {
  if (threadIdx.x < kWave) {
    double t = 0.0;
    for (int b = threadIdx.x; b < ntile; b += kWave) t += part[b];
    t = wsum(t);
    if (threadIdx.x == 0) *slot = t;
  }
  __syncthreads();
  const double v = *slot;
  __syncthreads();
  return v;
}

// Two such sums at once (one pass, one pair of barriers).
__device__ __forceinline__ void sum_parts2(const double* pa, const double* pb, int ntile, double* slot,
                                           double& a, double& b) {
  if (threadIdx.x < kWave) {
    double ta = 0.0, tb = 0.0;
    for (int k = threadIdx.x; k < ntile; k += kWave) {
      ta += pa[k];
      tb += pb[k];
    }
    ta = wsum(ta);
    tb = wsum(tb);
    if (threadIdx.x == 0) {
      slot[0] = ta;
      slot[1] = tb;
    }
  }
  __syncthreads();
  a = slot[0];
  b = slot[1];
  __syncthreads();
}

// the same for the one-thread-per-source start kernel
__device__ __forceinline__ double sum_parts_serial(const double* part, int ntile) {
  double t = 0.0;
  for (int b = 0; b < ntile; ++b) t += part[b];
  return t;
}

__global__ __launch_bounds__(kMT) void k_cgm_init(const double* __restrict__ kdia, int ldk, int nc,
                                                  int ns, int ntile, const double* __restrict__ rhs,
                                                  double* __restrict__ x, CgmState S) {
  __shared__ double red[kMT / kWave];
  int tile, j;
  if (!xcd_tile(ntile, tile, j)) return;
  const int i = tile * kMT + threadIdx.x;
  const bool live = i < nc && i != 0;
  const double dg = live ? kdia[13 * size_t(ldk) + i] : 0.0;
  const double dinv = dg > 0.0 ? 1.0 / dg : 0.0;
  const size_t o = size_t(j) * nc + i;
  const double r = live ? rhs[o] : 0.0;
  const double z = r * dinv;
  if (i < nc) {
    x[o] = 0.0;
    S.r[o] = r;
    S.p[o] = z;
  }
  const double rz = tile_sum<kMT / kWave>(r * z, red);
  const double rr = tile_sum<kMT / kWave>(r * r, red);
  if (threadIdx.x == 0) {
    S.part[(size_t(1) * ns + j) * ntile + tile] = rz;
    S.part[(size_t(2) * ns + j) * ntile + tile] = rr;
  }
}

// scalars of the initial residual (one thread per source)
__global__ void k_cgm_start(int ns, int ntile, int defl, CgmState S) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= ns) return;
  const double rz = sum_parts_serial(S.part + (size_t(1) * ns + j) * ntile, ntile) + (defl ? S.sy[j] : 0.0);
  const double bb = sum_parts_serial(S.part + (size_t(2) * ns + j) * ntile, ntile);
  S.scal[3 * j + 0] = rz;
  S.scal[3 * j + 1] = rz;
  S.scal[3 * j + 2] = bb;
  const int done = bb > 0.0 ? 0 : 1;
  S.flag[3 * j + 0] = done;
  S.flag[3 * j + 1] = done;
  S.flag[3 * j + 2] = 0;
}

// Two-level correction of the multi-launch solver, z = D^-1 r + Z E^-1 Z^T r:
// s = Z^T r by one workgroup per (aggregate, source), striding over the
// aggregate's vertex list in a fixed order; then y = E^-1 s and s.y by one
// workgroup per source (r.z = r.D^-1 r + s.y).  Sources already stopped are
// skipped when live_only is set.
__global__ __launch_bounds__(kMT) void k_cgm_aggsum(int nc, int ns, int par, int live_only, CoarseDefl d,
                                                    CgmState S) {
  __shared__ double red[kMT / kWave];
  const int a = blockIdx.x, j = blockIdx.y;
  if (live_only && S.flag[3 * j + par]) return;  // uniform over the workgroup
  const int* rows = d.arows + d.na + 1;
  const double* rj = S.r + size_t(j) * nc;
  double t = 0.0;
  for (int k = d.arows[a] + threadIdx.x; k < d.arows[a + 1]; k += kMT) t += rj[rows[k]];
  t = tile_sum<kMT / kWave>(t, red);
  if (threadIdx.x == 0) S.s[size_t(j) * 64 + a] = t;
}

// y = E^-1 s and s.y, one workgroup per source: thread (q, t) adds columns
// [16q, 16q + 16) of row t (E^-1 is symmetric, so column c is read across
// the lanes: one coalesced load a step, sixteen of them independent), and
// the four quarters are added in LDS in a fixed order.
__global__ __launch_bounds__(kMT) void k_cgm_ysolve(int ns, int par, int live_only, CoarseDefl d,
                                                    CgmState S) {
  __shared__ double part[kMT / kWave][kWave];
  const int j = blockIdx.x, t = threadIdx.x & (kWave - 1), q = threadIdx.x / kWave;
  if (live_only && S.flag[3 * j + par]) return;  // uniform over the workgroup
  const double* sj = S.s + size_t(j) * 64;
  double y = 0.0;
  if (t < d.na) {
#pragma unroll
    for (int cc = 0; cc < 16; ++cc) {
      const int c = q * 16 + cc;
      if (c < d.na) y += d.einv[c * d.na + t] * sj[c];
    }
  }
  part[q][t] = y;
  __syncthreads();
  if (q == 0) {
    y = part[0][t] + part[1][t] + part[2][t] + part[3][t];
    if (t < d.na) S.y[size_t(j) * 64 + t] = y;
    const double sy = wsum(t < d.na ? sj[t] * y : 0.0);
    if (t == 0) S.sy[j] = sy;
  }
}

// p += Z y after the initial residual (p = D^-1 r from the init kernel)
__global__ __launch_bounds__(kMT) void k_cgm_pcorr(const double* __restrict__ kdia, int ldk, int ncx, int ncy,
                                                   int nc, int ntile, CoarseDefl d, CgmState S) {
  int tile, j;
  if (!xcd_tile(ntile, tile, j)) return;
  const int i = tile * kMT + threadIdx.x;
  if (i >= nc || i == 0) return;
  if (!(kdia[13 * size_t(ldk) + i] > 0.0)) return;
  const int a = agg_index(d, i % ncx, (i / ncx) % ncy, i / (ncx * ncy));
  S.p[size_t(j) * nc + i] += S.y[size_t(j) * 64 + a];
}

__global__ __launch_bounds__(kMT) void k_cgm_spmv(const double* __restrict__ kdia, int ldk, int ncx,
                                                  int ncy, int ncz, int ns, int ntile, int par,
                                                  CgmState S) {
  __shared__ double red[kMT / kWave * kMG];
  const int nc = ncx * ncy * ncz;
  int tile, grp;
  if (!xcd_tile(ntile, tile, grp)) return;
  const int i = tile * kMT + threadIdx.x;
  const int j0 = grp * kMG;
  const bool live = i < nc && i != 0;
  const int x = i % ncx, y = (i / ncx) % ncy, z = i / (ncx * ncy);
  double k[27];
#pragma unroll
  for (int o = 0; o < 27; ++o) {
    const int dx = o % 3 - 1, dy = (o / 3) % 3 - 1, dz = o / 9 - 1;
    const bool in = live && x + dx >= 0 && x + dx < ncx && y + dy >= 0 && y + dy < ncy &&
                    z + dz >= 0 && z + dz < ncz && i + dx + ncx * (dy + ncy * dz) != 0;
    k[o] = in ? kdia[size_t(o) * ldk + i] : 0.0;
  }
  // The group's sources one after another without a barrier between them
  // (their loads overlap), then one reduction for all of their p.q.
  double pq[kMG];
#pragma unroll
  for (int jj = 0; jj < kMG; ++jj) {
    pq[jj] = 0.0;
    const int j = j0 + jj;
    if (j >= ns || S.flag[3 * j + par]) continue;  // uniform over the workgroup
    const double* pj = S.p + size_t(j) * nc;
    if (live) {
      double q = 0.0;
#pragma unroll
      for (int o = 0; o < 27; ++o) {
        const int off = (o % 3 - 1) + ncx * ((o / 3) % 3 - 1 + ncy * (o / 9 - 1));
        if (k[o] != 0.0) q += k[o] * pj[i + off];
      }
      S.q[size_t(j) * nc + i] = q;
      pq[jj] = pj[i] * q;
    }
  }
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
#pragma unroll
  for (int jj = 0; jj < kMG; ++jj) {
    pq[jj] = wsum(pq[jj]);
    if (lane == 0) red[wid * kMG + jj] = pq[jj];
  }
  __syncthreads();
  if (threadIdx.x < kMG) {
    const int j = j0 + threadIdx.x;
    if (j < ns && !S.flag[3 * j + par]) {
      double t = red[threadIdx.x];
      for (int w = 1; w < kMT / kWave; ++w) t += red[w * kMG + threadIdx.x];
      S.part[(size_t(0) * ns + j) * ntile + tile] = t;
    }
  }
}

__global__ __launch_bounds__(kMT) void k_cgm_update(const double* __restrict__ kdia, int ldk, int nc,
                                                    int ns, int ntile, int par,
                                                    double* __restrict__ x, CgmState S) {
  __shared__ double red[2 * (kMT / kWave)];
  __shared__ double slot;
  int tile, j;
  if (!xcd_tile(ntile, tile, j)) return;
  const int i = tile * kMT + threadIdx.x;
  if (S.flag[3 * j + par]) return;  // uniform over the workgroup
  const bool live = i < nc && i != 0;
  const size_t o = size_t(j) * nc + i;
  // the row's operands first, so that their loads are in flight while wave 0
  // sums the partials
  double pv = 0.0, qv = 0.0, rv = 0.0, xv = 0.0, dinv = 0.0;
  if (live) {
    const double dg = kdia[13 * size_t(ldk) + i];
    dinv = dg > 0.0 ? 1.0 / dg : 0.0;
    pv = S.p[o];
    qv = S.q[o];
    rv = S.r[o];
    xv = x[o];
  }
  const double pq = sum_parts(S.part + (size_t(0) * ns + j) * ntile, ntile, &slot);
  const double alpha = pq != 0.0 ? S.scal[3 * j + par] / pq : 0.0;
  double rz = 0.0, rr = 0.0;
  if (live) {
    x[o] = xv + alpha * pv;
    const double r = rv - alpha * qv;
    S.r[o] = r;
    rz = r * r * dinv;
    rr = r * r;
  }
  // both tile sums in one pass (waves added in a fixed order)
  rz = wsum(rz);
  rr = wsum(rr);
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  if (lane == 0) {
    red[2 * wid] = rz;
    red[2 * wid + 1] = rr;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double t = red[threadIdx.x];
    for (int w = 1; w < kMT / kWave; ++w) t += red[2 * w + threadIdx.x];
    S.part[(size_t(1 + threadIdx.x) * ns + j) * ntile + tile] = t;
  }
}

// it: number of this iteration (1-based, the same for every source)
__global__ __launch_bounds__(kMT) void k_cgm_pupdate(const double* __restrict__ kdia, int ldk, int ncx,
                                                     int ncy, int nc, int ns, int ntile, int par, int it,
                                                     double tol2, int maxit, int defl, CoarseDefl d,
                                                     CgmState S, int* status, unsigned long long* work) {
  __shared__ double slot[2];
  int tile, j;
  if (!xcd_tile(ntile, tile, j)) return;
  const int i = tile * kMT + threadIdx.x;
  const int nxt = par ^ 1;
  if (S.flag[3 * j + par]) {
    if (tile == 0 && threadIdx.x == 0) {
      S.flag[3 * j + nxt] = 1;
      S.scal[3 * j + nxt] = S.scal[3 * j + par];
    }
    return;
  }
  const bool live = i < nc && i != 0;
  const size_t o = size_t(j) * nc + i;
  // the row's operands first (in flight while wave 0 sums the partials)
  double rv = 0.0, pv = 0.0, dinv = 0.0, yv = 0.0;
  if (live) {
    const double dg = kdia[13 * size_t(ldk) + i];
    dinv = dg > 0.0 ? 1.0 / dg : 0.0;
    rv = S.r[o];
    pv = S.p[o];
    if (defl && dinv != 0.0) yv = S.y[size_t(j) * 64 + agg_index(d, i % ncx, (i / ncx) % ncy, i / (ncx * ncy))];
  }
  double rz, rr;
  sum_parts2(S.part + (size_t(1) * ns + j) * ntile, S.part + (size_t(2) * ns + j) * ntile, ntile, slot, rz, rr);
  if (defl) rz += S.sy[j];
  const bool conv = rr <= tol2 * S.scal[3 * j + 2];
  const bool bad = rr != rr || (!conv && it >= maxit);
  const bool stop = conv || bad;
  if (tile == 0 && threadIdx.x == 0) {
    S.flag[3 * j + nxt] = stop ? 1 : 0;
    S.scal[3 * j + nxt] = rz;
    if (stop) {
      atomicMax(status + kStCoarseMaxIt, it);
      if (bad) atomicAdd(status + kStCoarseNoconv, 1);
      const double b2 = S.scal[3 * j + 2];
      if (b2 > 0.0) note_residual(status, kStCoarseRes, rr / b2);
      if (work) atomicAdd(work, (unsigned long long)it * (unsigned long long)nc);
    }
  }
  if (stop || !live) return;
  const double rzo = S.scal[3 * j + par];
  const double beta = rzo != 0.0 ? rz / rzo : 0.0;
  S.p[o] = (rv * dinv + yv) + beta * pv;
}

constexpr int kBlock = 1024;

// LDS halo of the single-workgroup solver: the largest row shift of the
// stencil (no z-shift on a 2-D grid)
int coarse_pad(const int ncv[3]) { return 1 + ncv[0] + (ncv[2] > 1 ? ncv[0] * ncv[1] : 0); }

// RPT consecutive rows a thread (2, 4 or 6; at 8 rows a thread the strided
// layout measured faster: 35 against 39 us an iteration at 19^3 vertices)
int qm_rows(int ldk, int ncx) {
  (void)ncx;
  const int rpt = ldk / kBlock;
  return (rpt == 2 || rpt == 4 || rpt == 6) ? rpt : 0;
}

size_t pcg_lds_bytes(int ldk, int pad, int na, int qm = 0) {
  const size_t pn = qm ? size_t(qm) * (kBlock + 2 * (pad / qm + 2)) : size_t(ldk) + 2 * pad;
  // with aggregates: their list offsets (72 ints) and the LDS position of
  // every row (ldk ints)
  const size_t tab = na > 0 ? (72 + size_t(ldk) + 1) / 2 : 0;
  return (pn + 2 * (kBlock / kWave) * 4 + size_t(na) * na + 128 + tab) * sizeof(double);
}

size_t setup_lds_bytes(int na) { return 2 * size_t(na) * na * sizeof(double); }

}  // namespace

int coarse_ldk(int nc) {
  const int rpt = (nc + kBlock - 1) / kBlock;
  if (rpt > 16) return rpt * kBlock;  // large systems: no LDS staging, rows just padded
  const int r = rpt <= 1 ? 1 : rpt <= 2 ? 2 : rpt <= 4 ? 4 : rpt <= 6 ? 6 : rpt <= 8 ? 8 : 16;
  return r * kBlock;
}

bool coarse_is_large(const int ncv[3]) {
  const int nc = ncv[0] * ncv[1] * ncv[2];
  const int pad = coarse_pad(ncv);
  const int ldk = coarse_ldk(nc);
  // more than 8 rows a thread spill in the single-workgroup kernel, which
  // then runs slower than the multi-launch solver (measured 2.8x at 21^3)
  return nc > 8 * kBlock || pcg_lds_bytes(ldk, pad, 0, qm_rows(ldk, ncv[0])) > 160 * 1024;
}

size_t coarse_large_workspace(const int ncv[3], int ns) {
  const size_t nc = size_t(ncv[0]) * ncv[1] * ncv[2];
  const size_t ntile = (nc + kMT - 1) / kMT;
  return (3 * nc * ns + 3 * ntile * ns + 3 * size_t(ns) + 129 * size_t(ns)) * sizeof(double) +
         3 * size_t(ns) * sizeof(int);
}

hipError_t launch_coarse_pcg_large(const double* kdia, const int ncv[3], const double* rhs, double* x,
                                   int ns, double rtol, int maxit, const CoarseDefl* defl, void* workspace,
                                   int* host_flags, int* status, unsigned long long* work, hipStream_t s) {
  if (ns == 0) return hipSuccess;
  const int nc = ncv[0] * ncv[1] * ncv[2];
  const int ldk = coarse_ldk(nc);
  const int ntile = (nc + kMT - 1) / kMT;
  CgmState S;
  double* w = static_cast<double*>(workspace);
  S.r = w;
  S.p = S.r + size_t(ns) * nc;
  S.q = S.p + size_t(ns) * nc;
  S.part = S.q + size_t(ns) * nc;
  S.scal = S.part + size_t(3) * ntile * ns;
  S.s = S.scal + size_t(3) * ns;
  S.y = S.s + size_t(64) * ns;
  S.sy = S.y + size_t(64) * ns;
  S.flag = reinterpret_cast<int*>(S.sy + size_t(ns));
  const bool two = defl && defl->ok && defl->einv && defl->arows && defl->na <= 64;
  const CoarseDefl d = two ? *defl : CoarseDefl();
  const dim3 gt(xcd_grid(ntile, ns)), gs(xcd_grid(ntile, (ns + kMG - 1) / kMG)), ga(two ? d.na : 1, ns);
  hipLaunchKernelGGL(k_cgm_init, gt, dim3(kMT), 0, s, kdia, ldk, nc, ns, ntile, rhs, x, S);
  if (two) {
    hipLaunchKernelGGL(k_cgm_aggsum, ga, dim3(kMT), 0, s, nc, ns, 0, 0, d, S);
    hipLaunchKernelGGL(k_cgm_ysolve, dim3(ns), dim3(kMT), 0, s, ns, 0, 0, d, S);
    hipLaunchKernelGGL(k_cgm_pcorr, gt, dim3(kMT), 0, s, kdia, ldk, ncv[0], ncv[1], nc, ntile, d, S);
  }
  hipLaunchKernelGGL(k_cgm_start, dim3((ns + 255) / 256), dim3(256), 0, s, ns, ntile, two ? 1 : 0, S);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const double tol2 = rtol * rtol;
  // Phases are issued in chunks.  After each chunk the stop flags (a few
  // bytes) are copied to the host; the host checks them one chunk late, with
  // the next chunk already queued, so the GPU never waits for the host.  A
  // chunk queued after every source has stopped only runs early exits.
  constexpr int kChunk = 8;
  hipEvent_t ev[2] = {nullptr, nullptr};
  for (int k = 0; k < 2; ++k) {
    e = hipEventCreateWithFlags(&ev[k], hipEventDisableTiming);
    if (e != hipSuccess) {
      if (ev[0]) (void)hipEventDestroy(ev[0]);
      return e;
    }
  }
  int it = 0, par = 0, pending = -1, pending_par = 0, chunk = 0;
  auto all_stopped = [&](int buf, int fpar) {
    const int* f = host_flags + 3 * ns * buf;
    for (int j = 0; j < ns; ++j)
      if (f[3 * j + fpar] == 0) return false;
    return true;
  };
  while (e == hipSuccess) {
    if (it >= maxit) {
      // the last chunk is queued: wait for it and stop
      e = hipStreamSynchronize(s);
      break;
    }
    for (int c = 0; c < kChunk && it < maxit; ++c, ++it) {
      hipLaunchKernelGGL(k_cgm_spmv, gs, dim3(kMT), 0, s, kdia, ldk, ncv[0], ncv[1], ncv[2], ns, ntile,
                         par, S);
      hipLaunchKernelGGL(k_cgm_update, gt, dim3(kMT), 0, s, kdia, ldk, nc, ns, ntile, par, x, S);
      if (two) {
        hipLaunchKernelGGL(k_cgm_aggsum, ga, dim3(kMT), 0, s, nc, ns, par, 1, d, S);
        hipLaunchKernelGGL(k_cgm_ysolve, dim3(ns), dim3(kMT), 0, s, ns, par, 1, d, S);
      }
      hipLaunchKernelGGL(k_cgm_pupdate, gt, dim3(kMT), 0, s, kdia, ldk, ncv[0], ncv[1], nc, ns, ntile, par,
                         it + 1, tol2, maxit, two ? 1 : 0, d, S, status, work);
      par ^= 1;
    }
    e = hipGetLastError();
    if (e != hipSuccess) break;
    const int buf = chunk & 1;
    e = hipMemcpyAsync(host_flags + 3 * ns * buf, S.flag, sizeof(int) * 3 * ns, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipEventRecord(ev[buf], s);
    if (e != hipSuccess) break;
    if (pending >= 0) {
      e = hipEventSynchronize(ev[pending]);
      if (e != hipSuccess) break;
      if (all_stopped(pending, pending_par)) {
        e = hipStreamSynchronize(s);  // the chunk just queued runs early exits
        break;
      }
    }
    pending = buf;
    pending_par = par;
    ++chunk;
  }
  for (int k = 0; k < 2; ++k) (void)hipEventDestroy(ev[k]);
  return e;
}

CoarseDefl coarse_defl_plan_large(const int ncv[3]) {
  CoarseDefl d = coarse_defl_plan(ncv);
  d.ok = d.na >= 2 && setup_lds_bytes(d.na) <= 160 * 1024;
  return d;
}

CoarseDefl coarse_defl_plan(const int ncv[3]) {
  CoarseDefl d;
  for (int k = 0; k < 3; ++k) d.b[k] = std::min(4, std::max(1, ncv[k]));
  auto count = [&](int k) { return (ncv[k] + d.b[k] - 1) / d.b[k]; };
  for (;;) {
    for (int k = 0; k < 3; ++k) d.na3[k] = count(k);
    d.na = d.na3[0] * d.na3[1] * d.na3[2];
    if (d.na <= 64) break;
    int kmax = 0;
    for (int k = 1; k < 3; ++k)
      if (d.na3[k] > d.na3[kmax]) kmax = k;
    d.b[kmax] *= 2;
  }
  const int nc = ncv[0] * ncv[1] * ncv[2];
  const int pad = coarse_pad(ncv);
  d.ok = d.na >= 2 && pcg_lds_bytes(coarse_ldk(nc), pad, d.na, qm_rows(coarse_ldk(nc), ncv[0])) <= 160 * 1024 &&
         setup_lds_bytes(d.na) <= 160 * 1024;
  return d;
}

std::vector<int> coarse_defl_rows(const CoarseDefl& d, const int ncv[3]) {
  std::vector<int> out(size_t(d.na) + 1, 0);
  out.reserve(out.size() + size_t(ncv[0]) * ncv[1] * ncv[2]);
  for (int a = 0; a < d.na; ++a) {
    const int ax = a % d.na3[0], ay = (a / d.na3[0]) % d.na3[1], az = a / (d.na3[0] * d.na3[1]);
    const int x0 = ax * d.b[0], y0 = ay * d.b[1], z0 = az * d.b[2];
    const int x1 = std::min(x0 + d.b[0], ncv[0]), y1 = std::min(y0 + d.b[1], ncv[1]),
              z1 = std::min(z0 + d.b[2], ncv[2]);
    for (int z = z0; z < z1; ++z)
      for (int y = y0; y < y1; ++y)
        for (int x = x0; x < x1; ++x) out.push_back(x + ncv[0] * (y + ncv[1] * z));
    out[size_t(a) + 1] = int(out.size()) - (d.na + 1);
  }
  return out;
}

hipError_t launch_coarse_defl_setup(const double* kdia, const int ncv[3], const CoarseDefl& d,
                                    double* einv, int* status, hipStream_t s) {
  if (!d.ok) return hipErrorInvalidConfiguration;
  const int nc = ncv[0] * ncv[1] * ncv[2];
  const size_t lds = setup_lds_bytes(d.na);
  auto kern = k_coarse_defl_setup<kBlock>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       int(lds));
    if (e != hipSuccess) return e;
  }
  // E assembled into einv by one wave an aggregate, then inverted in place
  hipLaunchKernelGGL(k_coarse_defl_assemble, dim3(d.na), dim3(kWave), 0, s, kdia, coarse_ldk(nc), ncv[0],
                     ncv[1], ncv[2], d, einv);
  hipLaunchKernelGGL(kern, dim3(1), dim3(kBlock), lds, s, einv, d, einv, status);
  return hipGetLastError();
}

hipError_t launch_coarse_pcg(const double* kdia, const int ncv[3], const double* rhs, double* x,
                             int ncol, double rtol, int maxit, const CoarseDefl* defl, int* status,
                             unsigned long long* work, hipStream_t s) {
  if (ncol == 0) return hipSuccess;
  const int nc = ncv[0] * ncv[1] * ncv[2];
  const int pad = coarse_pad(ncv);
  const int ldk = coarse_ldk(nc);
  const bool use = defl && defl->ok && defl->einv && defl->arows;
  const CoarseDefl d = use ? *defl : CoarseDefl();
  const int qm = qm_rows(ldk, ncv[0]);
  const size_t lds = pcg_lds_bytes(ldk, pad, use ? d.na : 0, qm);
  if (lds > 160 * 1024) return hipErrorInvalidConfiguration;
  const int rpt = ldk / kBlock;
  auto go = [&](auto kern) -> hipError_t {
    if (lds > 64 * 1024) {
      hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         int(lds));
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3(ncol), dim3(kBlock), lds, s, kdia, ldk, ncv[0], ncv[1], ncv[2], rhs, x,
                       rtol, maxit, d, status, work);
    return hipGetLastError();
  };
#define MSFV_QM_CASE(R)                                                                                  \
  if (qm == R) {                                                                                        \
    if (ncv[0] % R == 0)                                                                                \
      return use ? go(k_coarse_pcg<kBlock, R, true, 1>) : go(k_coarse_pcg<kBlock, R, false, 1>);        \
    return use ? go(k_coarse_pcg<kBlock, R, true, 2>) : go(k_coarse_pcg<kBlock, R, false, 2>);          \
  }
  MSFV_QM_CASE(2)
  MSFV_QM_CASE(4)
  MSFV_QM_CASE(6)
#undef MSFV_QM_CASE
#define MSFV_PCG_CASE(R)                                                                          \
  if (rpt <= R) return use ? go(k_coarse_pcg<kBlock, R, true, 0>) : go(k_coarse_pcg<kBlock, R, false, 0>);
  MSFV_PCG_CASE(1)  // up to 1024 rows
  MSFV_PCG_CASE(8)  // 6145-8192 rows (2, 4 and 6 rows a thread take the consecutive layouts)
#undef MSFV_PCG_CASE
  return hipErrorInvalidConfiguration;
}

}  // namespace msfv
