// C ABI of the MSFV library (declared in include/msfv.h): problem state,
// stage sequencing on one HIP stream, and host-side bookkeeping of sources,
// receivers and electrode loads.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "kernels.hpp"
#include "msfv.h"
#include "plan.hpp"

namespace {

thread_local std::string g_last_error;

msfv_status fail(msfv_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

#define HIP_OK(expr)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return fail(e_ == hipErrorOutOfMemory ? MSFV_ENOMEM : MSFV_EDEVICE,                     \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                         \
  } while (0)

template <typename T>
struct DevBuf {
  T* ptr = nullptr;
  size_t n = 0;    // logical size
  size_t cap = 0;  // allocated size: a smaller request reuses the allocation
  ~DevBuf() { release(); }
  void release() {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    n = cap = 0;
  }
  // (Re)size; reallocates (which synchronises the device) only to grow.
  hipError_t alloc(size_t count) {
    if (count <= cap && ptr) {
      n = count;
      return hipSuccess;
    }
    release();
    n = count;
    if (count == 0) return hipSuccess;
    hipError_t e = hipMalloc(&ptr, count * sizeof(T));
    if (e == hipSuccess) cap = count;
    else n = 0;
    return e;
  }
  // Blocking upload: the host vector may be a temporary.
  hipError_t upload(const std::vector<T>& h, hipStream_t s) {
    hipError_t e = alloc(h.size());
    if (e != hipSuccess || h.empty()) return e;
    e = hipMemcpyAsync(ptr, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s);
  }
  size_t bytes() const { return n * sizeof(T); }
};

struct Columns {
  int count = 0;
  std::vector<int> ptr, cell;
  std::vector<double> val;
};

// Per-stage HIP events on the problem's stream (enabled by msfv_profile_enable).
struct Profiler {
  bool on = false;
  std::vector<hipEvent_t> pool;
  size_t next = 0;
  std::vector<std::tuple<int, hipEvent_t, hipEvent_t>> recs;
  hipEvent_t get() {
    if (next < pool.size()) return pool[next++];
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    pool.push_back(e);
    ++next;
    return e;
  }
  ~Profiler() {
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

}  // namespace

struct msfv_problem {
  msfv_config cfg{};
  hipStream_t stream = nullptr;
  msfv::Plan plan;
  msfv::GridInfo g{};
  Columns src, rec;
  bool electrodes_ready = false;
  bool have_forward = false;
  bool basis_ready = false;  // S_k holds the basis of some model (a forward has run)
  bool frozen = false;       // forwards keep S_k and rebuild A_k(m) only
  unsigned long long generation = 0;  // bumped whenever device buffers are (re)allocated

  // plan on the device
  DevBuf<msfv::EntDesc> d_edges, d_faces, d_blocks;
  DevBuf<int> d_prow, d_pcol, d_krow, d_kcol, d_kcptr, d_kcidx, d_kdslot, d_vrows;
  DevBuf<double> d_pval, d_kval, d_kdia, d_kent, d_inbuf, d_W;
  DevBuf<double> d_m;    // copy of the m of the last forward
  DevBuf<double> d_sig;  // exp of it
  DevBuf<int> d_status;

  // sources / receivers / electrodes
  DevBuf<int> d_rptr, d_rcell;
  DevBuf<double> d_rval;
  DevBuf<int> d_src_dst, d_src_ptr, d_src_pidx;
  DevBuf<double> d_src_w;
  DevBuf<int> d_rec_dst, d_rec_ptr, d_rec_pidx, d_rec_col;
  DevBuf<double> d_rec_w;
  DevBuf<int> d_ecell, d_erptr, d_eridx, d_esptr, d_esidx, d_eidx, d_eloc;
  DevBuf<double> d_erw, d_esw, d_sload;
  int nelec = 0, nsrc_slot = 0, nrec_slot = 0;

  // coarse vectors (column j contiguous) and data scratch
  // d_t holds t (Nc x Ns) followed by lambda (Nc x Ns), so that forward and
  // adjoint coarse problems can be solved in one launch of 2 Ns columns;
  // d_b holds their right-hand sides in the same order
  DevBuf<double> d_b, d_t, d_D, d_v;
  DevBuf<unsigned long long> d_work;
  // per-entity CG statistics of the four local stages (block fwd, block adj,
  // face fwd, face adj), at offsets ent_off[slot]
  DevBuf<int> d_ent_it;
  DevBuf<double> d_ent_res;  // 8 slots an entity: final (||r|| / ||b||)^2 of its local solves
  DevBuf<unsigned long long> d_ent_work;
  int ent_off[5] = {0, 0, 0, 0, 0};
  // two-level coarse preconditioner: aggregates and (Z^T A_k Z)^-1
  msfv::CoarseDefl defl;
  DevBuf<double> d_einv;
  DevBuf<int> d_arows;
  DevBuf<double> d_mu;  // adjoint local solutions of the wave kernels (per entity 8 x nu)
  // dual blocks split for launching: the full blocks of full_u^3 own cells
  // (geometry fixed at compile time) first, then the others
  DevBuf<int> d_blist;
  std::vector<int> h_blist;
  int full_u = 0, nfull = 0, nrest = 0;
  int edge_line = 0;  // longest closure line of an edge (cells)
  // faces in launch order: the full faces of face_u x face_u own cells
  // (nface_full, grouped by plane axis), then the others (nface_rest);
  // faces_one_launch: the others fit the same wave kernel
  DevBuf<int> d_flist;
  std::vector<int> h_flist;
  int face_u = 0, nface_full = 0, nface_rest = 0;
  bool faces_one_launch = false;
  // sensitivity passes (allocated on first use)
  DevBuf<double> d_dpval, d_dkent, d_dkval, d_dkdia, d_dt, d_fu, d_fz;
  DevBuf<int> d_ccptr, d_ccidx, d_cccell;  // column lists of S_k
  // large coarse systems: solver workspace and pinned stop flags
  DevBuf<double> d_cg_ws;
  int* h_flags = nullptr;
  int flags_cap = 0;  // sources h_flags has room for
  ~msfv_problem() {
    if (h_flags) (void)hipHostFree(h_flags);
  }
  Profiler prof;

  size_t workspace_bytes() const {
    return d_edges.bytes() + d_faces.bytes() + d_blocks.bytes() + d_prow.bytes() + d_pcol.bytes() +
           d_krow.bytes() + d_kcol.bytes() + d_kcptr.bytes() + d_kcidx.bytes() + d_kdslot.bytes() +
           d_vrows.bytes() + d_pval.bytes() + d_kval.bytes() + d_kdia.bytes() + d_kent.bytes() +
           d_inbuf.bytes() + d_W.bytes() +
           d_m.bytes() + d_sig.bytes() + d_b.bytes() + d_t.bytes() + d_D.bytes() + d_v.bytes() +
           d_sload.bytes() + d_einv.bytes() + d_arows.bytes() + d_cg_ws.bytes() + d_mu.bytes() + d_dpval.bytes() +
           d_dkent.bytes() + d_dkval.bytes() + d_dkdia.bytes() + d_dt.bytes() + d_fu.bytes() +
           d_fz.bytes() + d_ccptr.bytes() + d_ccidx.bytes() + d_cccell.bytes();
  }
};

namespace {

// Whether the coarse systems go to the multi-launch solver.
bool coarse_multi(const msfv_problem* p) {
  return p->cfg.coarse_precond == MSFV_COARSE_MULTI || msfv::coarse_is_large(p->plan.ncv);
}


// Launch ``expr`` as stage ``id``; with profiling on, bracket it by events.
#define STAGE(id, expr)                                                              \
  do {                                                                               \
    hipEvent_t e0_ = nullptr, e1_ = nullptr;                                         \
    if (p->prof.on) {                                                                \
      e0_ = p->prof.get();                                                           \
      e1_ = p->prof.get();                                                           \
      if (e0_) HIP_OK(hipEventRecord(e0_, p->stream));                               \
    }                                                                                \
    HIP_OK(expr);                                                                    \
    if (p->prof.on && e0_ && e1_) {                                                  \
      HIP_OK(hipEventRecord(e1_, p->stream));                                        \
      p->prof.recs.emplace_back(id, e0_, e1_);                                       \
    }                                                                                \
  } while (0)

msfv_status check_columns(const msfv_problem* p, int count, const int* ptr, const int* cell,
                          const double* val, Columns* out) {
  if (count < 0 || (count > 0 && (!ptr || !cell || !val)))
    return fail(MSFV_EINVAL, "sparse columns: null pointer or negative count");
  Columns c;
  c.count = count;
  c.ptr.assign(ptr, ptr + count + 1);
  if (c.ptr[0] != 0) return fail(MSFV_EINVAL, "sparse columns: ptr[0] must be 0");
  for (int j = 0; j < count; ++j)
    if (c.ptr[j + 1] < c.ptr[j]) return fail(MSFV_EINVAL, "sparse columns: ptr not monotone");
  const int nnz = c.ptr[count];
  c.cell.assign(cell, cell + nnz);
  c.val.assign(val, val + nnz);
  for (int e = 0; e < nnz; ++e) {
    if (c.cell[e] < 0 || c.cell[e] >= p->plan.ncell)
      return fail(MSFV_EINVAL, "sparse columns: cell index out of range");
    if (!std::isfinite(c.val[e])) return fail(MSFV_EINVAL, "sparse columns: non-finite value");
  }
  *out = std::move(c);
  return MSFV_OK;
}

// Electrode bookkeeping: direct adjoint loads, coarse right-hand-side
// gathers and per-entity electrode lists.
msfv_status build_electrodes(msfv_problem* p) {
  const msfv::Plan& P = p->plan;
  hipStream_t s = p->stream;
  const int ns = p->src.count, nr = p->rec.count;
  const int64_t nc = P.ncoarse;

  // coarse right-hand side of the forward: slot (j, vid) <- sum q * S_k[cell, vid]
  {
    std::map<std::pair<int, int>, std::vector<std::pair<int, double>>> slots;
    for (int j = 0; j < ns; ++j)
      for (int e = p->src.ptr[j]; e < p->src.ptr[j + 1]; ++e) {
        const int cell = p->src.cell[e];
        for (int q = P.prow[cell]; q < P.prow[cell + 1]; ++q)
          slots[{j, P.pcol[q]}].emplace_back(q, p->src.val[e]);
      }
    std::vector<int> dst, ptr{0}, pidx;
    std::vector<double> w;
    for (auto& kv : slots) {
      dst.push_back(int(kv.first.first * nc + kv.first.second));
      for (auto& ent : kv.second) {
        pidx.push_back(ent.first);
        w.push_back(ent.second);
      }
      ptr.push_back(int(pidx.size()));
    }
    p->nsrc_slot = int(dst.size());
    HIP_OK(p->d_src_dst.upload(dst, s));
    HIP_OK(p->d_src_ptr.upload(ptr, s));
    HIP_OK(p->d_src_pidx.upload(pidx, s));
    HIP_OK(p->d_src_w.upload(w, s));
  }
  // coarse right-hand side of the adjoint: slot vid <- sum_i v_ij * rval * S_k[cell, vid]
  {
    std::map<int, std::vector<std::tuple<int, double, int>>> slots;
    for (int i = 0; i < nr; ++i)
      for (int e = p->rec.ptr[i]; e < p->rec.ptr[i + 1]; ++e) {
        const int cell = p->rec.cell[e];
        for (int q = P.prow[cell]; q < P.prow[cell + 1]; ++q)
          slots[P.pcol[q]].emplace_back(q, p->rec.val[e], i);
      }
    std::vector<int> dst, ptr{0}, pidx, col;
    std::vector<double> w;
    for (auto& kv : slots) {
      dst.push_back(kv.first);
      for (auto& ent : kv.second) {
        pidx.push_back(std::get<0>(ent));
        w.push_back(std::get<1>(ent));
        col.push_back(std::get<2>(ent));
      }
      ptr.push_back(int(pidx.size()));
    }
    p->nrec_slot = int(dst.size());
    HIP_OK(p->d_rec_dst.upload(dst, s));
    HIP_OK(p->d_rec_ptr.upload(ptr, s));
    HIP_OK(p->d_rec_pidx.upload(pidx, s));
    HIP_OK(p->d_rec_col.upload(col, s));
    HIP_OK(p->d_rec_w.upload(w, s));
  }
  // electrodes: unique source/receiver cells that belong to an entity
  std::map<int, std::pair<std::vector<std::pair<int, double>>, std::vector<std::pair<int, double>>>> el;
  for (int i = 0; i < nr; ++i)
    for (int e = p->rec.ptr[i]; e < p->rec.ptr[i + 1]; ++e) el[p->rec.cell[e]].first.emplace_back(i, p->rec.val[e]);
  for (int j = 0; j < ns; ++j)
    for (int e = p->src.ptr[j]; e < p->src.ptr[j + 1]; ++e) el[p->src.cell[e]].second.emplace_back(j, p->src.val[e]);
  std::vector<int> ecell, erptr{0}, eridx, esptr{0}, esidx;
  std::vector<double> erw, esw;
  // per entity (kind, index) -> list of (electrode, own-cell index)
  std::map<std::pair<int, int>, std::vector<std::pair<int, int>>> per_ent;
  for (auto& kv : el) {
    int kind, idx;
    P.entity_of_cell(kv.first, &kind, &idx);
    if (kind == 0) continue;  // vertex cells: basis values do not depend on m
    const msfv::EntDesc* E = P.ent(kind, idx);
    const int cell = kv.first;
    const int x = cell % P.n[0], y = (cell / P.n[0]) % P.n[1], z = cell / (P.n[0] * P.n[1]);
    const int u = (x - E->ulo[0]) + E->uext[0] * ((y - E->ulo[1]) + E->uext[1] * (z - E->ulo[2]));
    const int eid = int(ecell.size());
    per_ent[{kind, idx}].emplace_back(eid, u);
    ecell.push_back(cell);
    for (auto& r : kv.second.first) {
      eridx.push_back(r.first);
      erw.push_back(r.second);
    }
    erptr.push_back(int(eridx.size()));
    for (auto& q : kv.second.second) {
      esidx.push_back(q.first);
      esw.push_back(q.second);
    }
    esptr.push_back(int(esidx.size()));
  }
  p->nelec = int(ecell.size());
  std::vector<int> eidx, eloc;
  for (auto* list : {&p->plan.edges, &p->plan.faces, &p->plan.blocks})
    for (auto& E : *list) E.eptr0 = E.eptr1 = 0;
  for (auto& kv : per_ent) {
    msfv::EntDesc* E = const_cast<msfv::EntDesc*>(P.ent(kv.first.first, kv.first.second));
    E->eptr0 = int(eidx.size());
    for (auto& q : kv.second) {
      eidx.push_back(q.first);
      eloc.push_back(q.second);
    }
    E->eptr1 = int(eidx.size());
  }
  if (eidx.empty()) {
    eidx.push_back(0);
    eloc.push_back(-1);
  }
  HIP_OK(p->d_ecell.upload(ecell, s));
  HIP_OK(p->d_erptr.upload(erptr, s));
  HIP_OK(p->d_eridx.upload(eridx.empty() ? std::vector<int>{0} : eridx, s));
  HIP_OK(p->d_erw.upload(erw.empty() ? std::vector<double>{0.0} : erw, s));
  HIP_OK(p->d_esptr.upload(esptr, s));
  HIP_OK(p->d_esidx.upload(esidx.empty() ? std::vector<int>{0} : esidx, s));
  HIP_OK(p->d_esw.upload(esw.empty() ? std::vector<double>{0.0} : esw, s));
  HIP_OK(p->d_eidx.upload(eidx, s));
  HIP_OK(p->d_eloc.upload(eloc, s));
  HIP_OK(p->d_sload.alloc(size_t(std::max(1, p->nelec)) * 8));
  HIP_OK(p->d_edges.upload(p->plan.edges, s));
  HIP_OK(p->d_faces.upload(p->plan.faces, s));
  HIP_OK(p->d_blocks.upload(p->plan.blocks, s));
  // receivers for the data gather
  HIP_OK(p->d_rptr.upload(p->rec.ptr, s));
  HIP_OK(p->d_rcell.upload(p->rec.cell.empty() ? std::vector<int>{0} : p->rec.cell, s));
  HIP_OK(p->d_rval.upload(p->rec.val.empty() ? std::vector<double>{0.0} : p->rec.val, s));
  // coarse vectors
  const size_t ncs = size_t(nc) * std::max(1, ns);
  // also the prolongation's scratch
  HIP_OK(p->d_b.alloc(std::max(size_t(nc) * msfv::prolong_ldt(ns), 2 * ncs)));
  HIP_OK(p->d_t.alloc(2 * ncs));
  HIP_OK(p->d_D.alloc(size_t(std::max(1, nr)) * std::max(1, ns)));
  HIP_OK(p->d_v.alloc(size_t(std::max(1, nr)) * std::max(1, ns)));
  if (coarse_multi(p)) {
    // room for the 2 Ns columns of a forward + adjoint solve
    HIP_OK(p->d_cg_ws.alloc(msfv::coarse_large_workspace(p->plan.ncv, 2 * std::max(1, ns)) / sizeof(double) + 1));
    if (p->flags_cap < 2 * ns) {  // grow only: freeing pinned memory synchronises the device
      if (p->h_flags) HIP_OK(hipHostFree(p->h_flags));
      p->h_flags = nullptr;
      p->flags_cap = 0;
      HIP_OK(hipHostMalloc(reinterpret_cast<void**>(&p->h_flags), sizeof(int) * 6 * 2 * std::max(1, ns)));
      p->flags_cap = 2 * std::max(1, ns);
    }
  }
  HIP_OK(hipStreamSynchronize(s));  // host vectors above are temporaries
  p->electrodes_ready = true;
  ++p->generation;
  return MSFV_OK;
}

// lambda (the adjoint coarse coefficients) sits after t in d_t
double* lam_ptr(msfv_problem* p) { return p->d_t.ptr + size_t(p->plan.ncoarse) * std::max(1, p->src.count); }

// Workgroups go round-robin over the eight XCDs (workgroup k to XCD k mod 8),
// each with its own L2.  The launch order of a list of entities deals them so
// that XCD x runs the x-th contiguous run of the list: neighbouring entities,
// which read the same lower-dimensional rows and the same m on their shared
// closure cells and write S_k rows into the same lines, meet in one L2.
std::vector<int> deal_over_xcds(const std::vector<int>& list) {
  const int nb = int(list.size()), q = nb / 8, r = nb % 8;
  std::vector<int> dealt(list.size());
  int start = 0;
  for (int x = 0; x < 8; ++x) {
    const int len = q + (x < r ? 1 : 0);
    for (int j = 0; j < len; ++j) dealt[size_t(8) * j + x] = list[size_t(start) + j];
    start += len;
  }
  return dealt;
}

msfv::LocalParams base_params(msfv_problem* p) {
  msfv::LocalParams lp;
  lp.g = p->g;
  lp.m = p->d_m.ptr;
  lp.sig = p->d_sig.ptr;
  lp.prow = p->d_prow.ptr;
  lp.pcol = p->d_pcol.ptr;
  lp.pval = p->d_pval.ptr;
  lp.kent = p->d_kent.ptr;
  lp.rtol = p->cfg.local_rtol;
  lp.maxit = p->cfg.local_maxit;
  lp.status = p->d_status.ptr;
  lp.sig_cap = p->plan.max_closure;
  lp.t = p->d_t.ptr;
  lp.lam = lam_ptr(p);
  lp.ncoarse = int(p->plan.ncoarse);
  lp.ns = p->src.count;
  lp.inbuf = p->d_inbuf.ptr;
  lp.outbuf = p->d_inbuf.ptr;
  lp.eidx = p->d_eidx.ptr;
  lp.eloc = p->d_eloc.ptr;
  lp.sload = p->d_sload.ptr;
  lp.W = p->d_W.ptr;
  return lp;
}

// Route the per-entity statistics of local stage ``slot`` (0 block fwd,
// 1 block adj, 2 face fwd, 3 face adj).
void set_stats(msfv_problem* p, msfv::LocalParams& lp, int slot) {
  lp.ent_it = p->d_ent_it.ptr + p->ent_off[slot];
  lp.ent_res = p->d_ent_res.ptr + size_t(8) * p->ent_off[slot];
  lp.ent_work = p->prof.on ? p->d_ent_work.ptr + p->ent_off[slot] : nullptr;
}

void set_caps(msfv::LocalParams& lp, const msfv::Plan::Caps& c, int nu_cap) {
  lp.nu_cap = nu_cap;
  lp.sig_cap = c.closure;
  lp.lane_cap = c.lane;
  lp.col_cap = c.col;
  lp.nc_cap = c.nc;
  lp.plane_cap = c.plane;
}

// Coarse solves of the ns columns of rhs with the configured preconditioner.
// ncol columns (default: one a source), column j at rhs + j Nc and x + j Nc
hipError_t coarse_solve(msfv_problem* p, const double* rhs, double* x, unsigned long long* work,
                        hipStream_t s, int ncol = -1) {
  const msfv::Plan& P = p->plan;
  if (ncol < 0) ncol = p->src.count;
  if (coarse_multi(p))
    return msfv::launch_coarse_pcg_large(p->d_kdia.ptr, P.ncv, rhs, x, ncol, p->cfg.coarse_rtol,
                                         p->cfg.coarse_maxit, p->defl.ok ? &p->defl : nullptr,
                                         p->d_cg_ws.ptr, p->h_flags, p->d_status.ptr, work, s);
  return msfv::launch_coarse_pcg(p->d_kdia.ptr, P.ncv, rhs, x, ncol, p->cfg.coarse_rtol,
                                 p->cfg.coarse_maxit, p->defl.ok ? &p->defl : nullptr,
                                 p->d_status.ptr, work, s);
}

// Launch caps of the full dual blocks of u^3 own cells (whatever the
// other blocks of the grid are).
void full_caps(msfv::LocalParams& lp, int u) {
  lp.nu_cap = u * u * u;
  lp.sig_cap = (u + 2) * (u + 2) * (u + 2);
  lp.lane_cap = u * u;
  lp.col_cap = u;
  lp.nc_cap = 8;
  lp.plane_cap = msfv::wave_plane(u, u) * u;
}

// Local solves of the dual blocks: the full blocks through the bodies
// specialised for their shape, the others through the general ones; the
// forward in one launch where the others fit the same wave kernel, else in
// two (the adjoint always in two: its two bodies in one kernel spill).
hipError_t launch_blocks(msfv_problem* p, const msfv::LocalParams& lp, bool adj, hipStream_t s) {
  if (!adj && p->nfull > 0 && p->nrest > 0 && msfv::wave_path_fits(lp) && lp.nc_cap <= 8 &&
      (p->full_u == 7 || lp.col_cap <= 3)) {
    msfv::LocalParams b = lp;
    b.ent_list = p->d_blist.ptr;
    b.nent = p->nfull + p->nrest;
    return msfv::launch_wave_blocks(b, p->full_u, s);
  }
  if (p->nfull > 0) {
    msfv::LocalParams f = lp;
    full_caps(f, p->full_u);
    f.ent_list = p->d_blist.ptr;
    f.nent = p->nfull;
    const hipError_t e = msfv::launch_wave_full(f, p->full_u, adj, s);
    if (e != hipSuccess) return e;
  }
  if (p->nrest > 0) {
    msfv::LocalParams r = lp;
    r.ent_list = p->d_blist.ptr + p->nfull;
    r.nent = p->nrest;
    return adj ? msfv::launch_local_adj(r, 0, s) : msfv::launch_local_fwd(r, 0, s);
  }
  return hipSuccess;
}

// Launch caps of the full faces of u x u own cells.
void face_caps(msfv::LocalParams& lp, int u) {
  lp.nu_cap = u * u;
  lp.sig_cap = (u + 2) * (u + 2);
  lp.lane_cap = u * u;
  lp.col_cap = 1;
  lp.nc_cap = 4;
  lp.plane_cap = msfv::wave_plane(u, u);
}

// Local solves of the faces: the full faces through bodies specialised for
// their shape, in one launch with the others where those fit the same wave
// kernel, else the others through the general kernels.
hipError_t launch_faces(msfv_problem* p, const msfv::LocalParams& lp, bool adj, hipStream_t s) {
  if (p->nface_full > 0 && p->faces_one_launch) return msfv::launch_wave_faces(lp, p->face_u, adj, s);
  if (p->nface_full > 0) {
    msfv::LocalParams f = lp;
    face_caps(f, p->face_u);
    f.nent = p->nface_full;
    const hipError_t e = msfv::launch_wave_faces(f, p->face_u, adj, s);
    if (e != hipSuccess) return e;
  }
  if (p->nface_rest > 0) {
    msfv::LocalParams r = lp;
    r.ent_list = p->d_flist.ptr + p->nface_full;
    r.nent = p->nface_rest;
    return adj ? msfv::launch_local_adj(r, 0, s) : msfv::launch_local_fwd(r, 0, s);
  }
  return hipSuccess;
}

msfv_status ensure_ready(msfv_problem* p) {
  if (p->src.count <= 0) return fail(MSFV_ESTATE, "no sources set");
  if (p->rec.count <= 0) return fail(MSFV_ESTATE, "no receivers set");
  if (!p->electrodes_ready) return build_electrodes(p);
  return MSFV_OK;
}

// Parameters of the local stages.  kind 1 edges, 2 faces (or the dual
// blocks of a 2-D grid), 3 dual blocks; adj selects the adjoint variant.
msfv::LocalParams local_params(msfv_problem* p, int kind, bool adj) {
  const msfv::Plan& P = p->plan;
  const bool lagrange = p->cfg.bc_mode == MSFV_BC_LAGRANGE;
  msfv::LocalParams lp = base_params(p);
  lp.lagrange = lagrange ? 1 : 0;
  if (kind == 1) {
    lp.ents = p->d_edges.ptr;
    lp.nent = int(P.edges.size());
    lp.line_cap = p->edge_line;
    return lp;
  }
  if (kind == 2) {
    lp.ents = p->d_faces.ptr;
    lp.ent_list = p->d_flist.ptr;
    lp.nent = int(P.faces.size());
    set_caps(lp, P.caps_face, P.max_nu_face);
    if (adj) {
      lp.mu_scratch = p->d_mu.ptr;
      lp.recv = p->d_edges.ptr;
      lp.push = lagrange ? 0 : 1;
      lp.solve_adj = (lagrange && P.dim == 3) ? 0 : 1;
      set_stats(p, lp, 3);
    } else {
      lp.prescribe = (lagrange && P.dim == 3) ? 1 : 0;
      set_stats(p, lp, 2);
    }
    return lp;
  }
  lp.ents = p->d_blocks.ptr;
  lp.nent = int(P.blocks.size());
  set_caps(lp, P.caps_block, P.max_nu_block);
  if (adj) {
    lp.mu_scratch = p->d_mu.ptr;
    lp.recv = p->d_faces.ptr;
    lp.push = lagrange ? 0 : 1;
    lp.solve_adj = 1;
    set_stats(p, lp, 1);
  } else {
    set_stats(p, lp, 0);
  }
  return lp;
}

// Forward, in three parts: the model of the call, the local solves (or the
// frozen basis's energy blocks), and the Galerkin coarse problem with the
// data.  A batch runs the middle part of many problems in shared launches.
msfv_status fwd_begin(msfv_problem* p, const double* m) {
  msfv_status st = ensure_ready(p);
  if (st != MSFV_OK) return st;
  const msfv::Plan& P = p->plan;
  hipStream_t s = p->stream;
  HIP_OK(msfv::launch_zero(p->d_status.ptr, sizeof(int) * msfv::kStCount, s));
  HIP_OK(msfv::launch_zero(p->d_ent_it.ptr, p->d_ent_it.bytes(), s));
  HIP_OK(msfv::launch_zero(p->d_ent_res.ptr, p->d_ent_res.bytes(), s));
  STAGE(MSFV_STAGE_COPY_M,
        msfv::launch_prep_model(p->d_m.ptr, p->d_sig.ptr, m, P.ncell, p->d_status.ptr, s));
  return MSFV_OK;
}

msfv_status fwd_local(msfv_problem* p) {
  const msfv::Plan& P = p->plan;
  hipStream_t s = p->stream;
  const bool lagrange = p->cfg.bc_mode == MSFV_BC_LAGRANGE;
  if (p->frozen) {
    // fixed basis (eq. optredfixed): S_k stays, A_k(m) = S_k^T A(m) S_k from
    // energy blocks over each entity's fluxes at the current m
    msfv::LocalParams lp = local_params(p, 1, false);
    lp.nc_cap = 2;
    STAGE(MSFV_STAGE_EDGE_FWD, msfv::launch_energy_frozen(lp, s));
    lp = local_params(p, 2, false);
    STAGE(MSFV_STAGE_FACE_FWD, msfv::launch_energy_frozen(lp, s));
    if (P.dim == 3) {
      lp = local_params(p, 3, false);
      STAGE(MSFV_STAGE_BLOCK_FWD, msfv::launch_energy_frozen(lp, s));
    }
    return MSFV_OK;
  }
  msfv::LocalParams lp = local_params(p, 1, false);
  STAGE(MSFV_STAGE_EDGE_FWD, msfv::launch_edge_fwd(lp, lagrange ? 1 : 0, s));
  lp = local_params(p, 2, false);
  STAGE(MSFV_STAGE_FACE_FWD, launch_faces(p, lp, false, s));
  if (P.dim == 3) {
    lp = local_params(p, 3, false);
    STAGE(MSFV_STAGE_BLOCK_FWD, launch_blocks(p, lp, false, s));
  }
  return MSFV_OK;
}

// Galerkin operator, coarse preconditioner and the forward right-hand sides
// S_k^T q_j (columns 0 .. Ns-1 of d_b); ncol_zero columns of d_b cleared.
msfv_status coarse_prep(msfv_problem* p, int ncol_zero) {
  const msfv::Plan& P = p->plan;
  hipStream_t s = p->stream;
  STAGE(MSFV_STAGE_KASSEMBLE,
        msfv::launch_kassemble(p->d_kcptr.ptr, p->d_kcidx.ptr, p->d_kdslot.ptr, p->d_kent.ptr,
                               p->d_kval.ptr, p->d_kdia.ptr, int(P.kcol.size()), s));
  if (p->defl.ok)
    STAGE(MSFV_STAGE_COARSE_SETUP,
          msfv::launch_coarse_defl_setup(p->d_kdia.ptr, P.ncv, p->defl, p->d_einv.ptr,
                                         p->d_status.ptr, s));
  const int nc = int(P.ncoarse);
  HIP_OK(msfv::launch_zero(p->d_b.ptr, sizeof(double) * size_t(nc) * ncol_zero, s));
  STAGE(MSFV_STAGE_COARSE_RHS,
        msfv::launch_gather_slots(p->d_src_dst.ptr, p->d_src_ptr.ptr, p->d_src_pidx.ptr,
                                  p->d_src_w.ptr, nullptr, nullptr, 0, p->d_pval.ptr, p->d_b.ptr,
                                  p->nsrc_slot, 1, nc, s));
  return MSFV_OK;
}

// D = Rx^T S_k t (and u = S_k t) from the solved t
msfv_status fwd_data(msfv_problem* p, double* d_out, double* u_out) {
  const msfv::Plan& P = p->plan;
  hipStream_t s = p->stream;
  const int ns = p->src.count, nr = p->rec.count;
  const int nc = int(P.ncoarse);
  STAGE(MSFV_STAGE_DATA,
        msfv::launch_data(p->d_rptr.ptr, p->d_rcell.ptr, p->d_rval.ptr, nr, ns, p->d_prow.ptr,
                          p->d_pcol.ptr, p->d_pval.ptr, p->d_t.ptr, nc, d_out, s));
  if (u_out)
    STAGE(MSFV_STAGE_PROLONG,
          msfv::launch_prolong(p->d_prow.ptr, p->d_pcol.ptr, p->d_pval.ptr, p->d_t.ptr, P.ncv, ns,
                               P.ncell, u_out, p->d_b.ptr, s));
  p->have_forward = true;
  p->basis_ready = true;
  return MSFV_OK;
}

msfv_status fwd_end(msfv_problem* p, double* d_out, double* u_out) {
  hipStream_t s = p->stream;
  msfv_status st = coarse_prep(p, p->src.count);
  if (st != MSFV_OK) return st;
  STAGE(MSFV_STAGE_COARSE_FWD,
        coarse_solve(p, p->d_b.ptr, p->d_t.ptr, p->d_work.ptr + 4, s));
  return fwd_data(p, d_out, u_out);
}

msfv_status forward_impl(msfv_problem* p, const double* m, double* d_out, double* u_out) {
  msfv_status st = fwd_begin(p, m);
  if (st == MSFV_OK) st = fwd_local(p);
  if (st == MSFV_OK) st = fwd_end(p, d_out, u_out);
  return st;
}

// J^T v in three parts: the adjoint coarse problem and the direct electrode
// loads, the local adjoint sweeps (blocks, faces, edges), and g.
// The adjoint right-hand sides S_k^T Rx v_j into rhs (Ns columns, cleared
// by the caller).
msfv_status adj_rhs(msfv_problem* p, const double* v, double* rhs) {
  const msfv::Plan& P = p->plan;
  hipStream_t s = p->stream;
  const int ns = p->src.count, nr = p->rec.count;
  const int nc = int(P.ncoarse);
  STAGE(MSFV_STAGE_ADJ_RHS,
        msfv::launch_gather_slots(p->d_rec_dst.ptr, p->d_rec_ptr.ptr, p->d_rec_pidx.ptr,
                                  p->d_rec_w.ptr, p->d_rec_col.ptr, v, nr, p->d_pval.ptr, rhs,
                                  p->nrec_slot, ns, nc, s));
  return MSFV_OK;
}

msfv_status adj_sload(msfv_problem* p, const double* v) {
  const msfv::Plan& P = p->plan;
  hipStream_t s = p->stream;
  const int ns = p->src.count, nr = p->rec.count;
  const int nc = int(P.ncoarse);
  STAGE(MSFV_STAGE_SLOAD,
        msfv::launch_sload(p->nelec, p->d_ecell.ptr, p->d_erptr.ptr, p->d_eridx.ptr, p->d_erw.ptr,
                           p->d_esptr.ptr, p->d_esidx.ptr, p->d_esw.ptr, p->d_prow.ptr, p->d_pcol.ptr,
                           p->d_t.ptr, lam_ptr(p), v, nc, ns, nr, p->d_sload.ptr, s));
  return MSFV_OK;
}

msfv_status adj_begin(msfv_problem* p, const double* v) {
  if (!p->have_forward) return fail(MSFV_ESTATE, "msfv_jtv called before msfv_forward");
  hipStream_t s = p->stream;
  const int nc = int(p->plan.ncoarse);
  HIP_OK(msfv::launch_zero(p->d_b.ptr, sizeof(double) * size_t(nc) * p->src.count, s));
  msfv_status st = adj_rhs(p, v, p->d_b.ptr);
  if (st != MSFV_OK) return st;
  STAGE(MSFV_STAGE_COARSE_ADJ,
        coarse_solve(p, p->d_b.ptr, lam_ptr(p), p->d_work.ptr + 5, s));
  return adj_sload(p, v);
}

// Forward and J^T v for a v given up front (not derived from this forward's
// D): the adjoint coarse problem A_k lambda_j = S_k^T Rx v_j needs only A_k,
// S_k and v, so its right-hand sides are gathered beside the forward's and
// both sets are solved in one launch of 2 Ns columns (t, then lambda).  Each
// column's iteration is the same as in separate solves, so the results are
// the same bit for bit.
msfv_status fwd_adj_coarse(msfv_problem* p, const double* v, double* d_out) {
  hipStream_t s = p->stream;
  const int ns = p->src.count;
  const size_t nc = size_t(p->plan.ncoarse);
  msfv_status st = coarse_prep(p, 2 * ns);
  if (st == MSFV_OK) st = adj_rhs(p, v, p->d_b.ptr + nc * ns);
  if (st != MSFV_OK) return st;
  STAGE(MSFV_STAGE_COARSE_FWD,
        coarse_solve(p, p->d_b.ptr, p->d_t.ptr, p->d_work.ptr + 4, s, 2 * ns));
  st = fwd_data(p, d_out, nullptr);
  if (st == MSFV_OK) st = adj_sload(p, v);
  return st;
}

msfv_status adj_local(msfv_problem* p) {
  const msfv::Plan& P = p->plan;
  hipStream_t s = p->stream;
  const bool lagrange = p->cfg.bc_mode == MSFV_BC_LAGRANGE;
  msfv::LocalParams lp;
  if (P.dim == 3) {
    lp = local_params(p, 3, true);
    STAGE(MSFV_STAGE_BLOCK_ADJ, launch_blocks(p, lp, true, s));
  }
  lp = local_params(p, 2, true);
  STAGE(MSFV_STAGE_FACE_ADJ, launch_faces(p, lp, true, s));
  lp = local_params(p, 1, true);
  STAGE(MSFV_STAGE_EDGE_ADJ, msfv::launch_edge_adj(lp, lagrange ? 1 : 0, s));
  return MSFV_OK;
}

msfv_status adj_end(msfv_problem* p, double* g_out) {
  hipStream_t s = p->stream;
  STAGE(MSFV_STAGE_GFINAL, msfv::launch_gfinal(p->d_sig.ptr, p->d_W.ptr, p->g, p->plan.ncell, g_out, s));
  return MSFV_OK;
}

msfv_status jtv_impl(msfv_problem* p, const double* v, double* g_out) {
  msfv_status st = adj_begin(p, v);
  if (st == MSFV_OK) st = adj_local(p);
  if (st == MSFV_OK) st = adj_end(p, g_out);
  return st;
}


// ---- sensitivities: forward-mode J dm and the fixed-basis variants ----------

msfv_status sens_ready_alloc(msfv_problem* p) {
  const msfv::Plan& P = p->plan;
  const size_t ncs = size_t(P.ncoarse) * std::max(1, p->src.count);
  HIP_OK(p->d_dt.alloc(ncs));
  return MSFV_OK;
}

msfv_status sens_ready(msfv_problem* p) {
  if (!p->have_forward) return fail(MSFV_ESTATE, "sensitivity call before msfv_forward");
  return sens_ready_alloc(p);
}

msfv_status fine_ready(msfv_problem* p) {
  const msfv::Plan& P = p->plan;
  const size_t n = size_t(P.ncell) * std::max(1, p->src.count);
  HIP_OK(p->d_fu.alloc(n));
  HIP_OK(p->d_fz.alloc(n));
  if (!p->d_ccptr.ptr) {  // column lists of S_k (static structure), in increasing cell order
    const int nc = int(P.ncoarse);
    std::vector<int> cptr(nc + 1, 0), cidx(P.pcol.size()), ccell(P.pcol.size());
    for (int c : P.pcol) ++cptr[c + 1];
    for (int v = 0; v < nc; ++v) cptr[v + 1] += cptr[v];
    std::vector<int> fill(cptr.begin(), cptr.end() - 1);
    for (int64_t i = 0; i < P.ncell; ++i)
      for (int e = P.prow[i]; e < P.prow[i + 1]; ++e) {
        const int k = fill[P.pcol[e]]++;
        cidx[k] = e;
        ccell[k] = int(i);
      }
    HIP_OK(p->d_ccptr.upload(cptr, p->stream));
    HIP_OK(p->d_ccidx.upload(cidx, p->stream));
    HIP_OK(p->d_cccell.upload(ccell, p->stream));
  }
  return MSFV_OK;
}

// J_k dm for the adaptive basis (eq. sensred in forward mode with the basis
// tangent of Sec. 4.5): dD = Rx^T (dS t + S dt), A_k dt = dS^T q - dA_k t.
msfv_status jvp_impl(msfv_problem* p, const double* dm, double* dd_out) {
  msfv_status st = sens_ready(p);
  if (st != MSFV_OK) return st;
  const msfv::Plan& P = p->plan;
  hipStream_t s = p->stream;
  const bool lagrange = p->cfg.bc_mode == MSFV_BC_LAGRANGE;
  const int ns = p->src.count, nr = p->rec.count, nc = int(P.ncoarse);
  if (!p->d_dpval.ptr) {
    HIP_OK(p->d_dpval.alloc(P.pcol.size()));
    HIP_OK(hipMemsetAsync(p->d_dpval.ptr, 0, p->d_dpval.bytes(), s));  // vertex rows stay 0
    HIP_OK(p->d_dkent.alloc(std::max<int64_t>(1, P.kent_size)));
    HIP_OK(p->d_dkval.alloc(std::max<size_t>(1, P.kcol.size())));
    HIP_OK(p->d_dkdia.alloc(p->d_kdia.n));
    HIP_OK(hipMemsetAsync(p->d_dkdia.ptr, 0, p->d_dkdia.bytes(), s));
  }
  HIP_OK(msfv::launch_zero(p->d_status.ptr, sizeof(int) * msfv::kStCount, s));
  HIP_OK(msfv::launch_check_finite(dm, P.ncell, p->d_status.ptr, s));
  msfv::LocalParams lp = base_params(p);
  lp.dm = dm;
  lp.dpval = p->d_dpval.ptr;
  lp.kent = p->d_dkent.ptr;
  lp.ents = p->d_edges.ptr;
  lp.nent = int(P.edges.size());
  HIP_OK(msfv::launch_edge_tan(lp, lagrange ? 1 : 0, s));
  lp.ents = p->d_faces.ptr;
  lp.nent = int(P.faces.size());
  set_caps(lp, P.caps_face, P.max_nu_face);
  lp.prescribe = (lagrange && P.dim == 3) ? 1 : 0;
  HIP_OK(msfv::launch_local_tan(lp, s));
  if (P.dim == 3) {
    lp.ents = p->d_blocks.ptr;
    lp.nent = int(P.blocks.size());
    set_caps(lp, P.caps_block, P.max_nu_block);
    lp.prescribe = 0;
    HIP_OK(msfv::launch_local_tan(lp, s));
  }
  HIP_OK(msfv::launch_kassemble(p->d_kcptr.ptr, p->d_kcidx.ptr, p->d_kdslot.ptr, p->d_dkent.ptr,
                                p->d_dkval.ptr, p->d_dkdia.ptr, int(P.kcol.size()), s));
  HIP_OK(msfv::launch_zero(p->d_b.ptr, sizeof(double) * size_t(nc) * ns, s));
  HIP_OK(msfv::launch_gather_slots(p->d_src_dst.ptr, p->d_src_ptr.ptr, p->d_src_pidx.ptr, p->d_src_w.ptr,
                                   nullptr, nullptr, 0, p->d_dpval.ptr, p->d_b.ptr, p->nsrc_slot, 1, nc, s));
  HIP_OK(msfv::launch_coarse_dk_sub(p->d_dkdia.ptr, msfv::coarse_ldk(nc), P.ncv, ns, p->d_t.ptr,
                                    p->d_b.ptr, s));
  HIP_OK(coarse_solve(p, p->d_b.ptr, p->d_dt.ptr, nullptr, s));
  HIP_OK(msfv::launch_data(p->d_rptr.ptr, p->d_rcell.ptr, p->d_rval.ptr, nr, ns, p->d_prow.ptr,
                           p->d_pcol.ptr, p->d_dpval.ptr, p->d_t.ptr, nc, dd_out, s, 0));
  HIP_OK(msfv::launch_data(p->d_rptr.ptr, p->d_rcell.ptr, p->d_rval.ptr, nr, ns, p->d_prow.ptr,
                           p->d_pcol.ptr, p->d_pval.ptr, p->d_dt.ptr, nc, dd_out, s, 1));
  return MSFV_OK;
}

// J dm with the basis held fixed (eq. senssimple): dD = -Rx^T S A_k^-1 S^T (dA u).
msfv_status jvp_fixed_impl(msfv_problem* p, const double* dm, double* dd_out) {
  msfv_status st = sens_ready(p);
  if (st == MSFV_OK) st = fine_ready(p);
  if (st != MSFV_OK) return st;
  const msfv::Plan& P = p->plan;
  hipStream_t s = p->stream;
  const int ns = p->src.count, nr = p->rec.count, nc = int(P.ncoarse);
  HIP_OK(msfv::launch_zero(p->d_status.ptr, sizeof(int) * msfv::kStCount, s));
  HIP_OK(msfv::launch_check_finite(dm, P.ncell, p->d_status.ptr, s));
  HIP_OK(msfv::launch_prolong(p->d_prow.ptr, p->d_pcol.ptr, p->d_pval.ptr, p->d_t.ptr, P.ncv, ns, P.ncell,
                              p->d_fu.ptr, p->d_b.ptr, s));
  HIP_OK(msfv::launch_dAu(p->d_m.ptr, dm, p->g, P.ncell, ns, p->d_fu.ptr, p->d_fz.ptr, s));
  HIP_OK(msfv::launch_restrict(p->d_ccptr.ptr, p->d_ccidx.ptr, p->d_cccell.ptr, p->d_pval.ptr, p->d_fz.ptr,
                               nc, ns, P.ncell, -1.0, p->d_b.ptr, s));
  HIP_OK(coarse_solve(p, p->d_b.ptr, p->d_dt.ptr, nullptr, s));
  HIP_OK(msfv::launch_data(p->d_rptr.ptr, p->d_rcell.ptr, p->d_rval.ptr, nr, ns, p->d_prow.ptr,
                           p->d_pcol.ptr, p->d_pval.ptr, p->d_dt.ptr, nc, dd_out, s, 0));
  return MSFV_OK;
}

// J^T v with the basis held fixed: lambda = A_k^-1 S^T Rx v,
// g = -grad_m sum_j (S lambda_j)^T A(m) u_j.
msfv_status jtv_fixed_impl(msfv_problem* p, const double* v, double* g_out) {
  msfv_status st = sens_ready(p);
  if (st == MSFV_OK) st = fine_ready(p);
  if (st != MSFV_OK) return st;
  const msfv::Plan& P = p->plan;
  hipStream_t s = p->stream;
  const int ns = p->src.count, nr = p->rec.count, nc = int(P.ncoarse);
  HIP_OK(msfv::launch_zero(p->d_b.ptr, sizeof(double) * size_t(nc) * ns, s));
  HIP_OK(msfv::launch_gather_slots(p->d_rec_dst.ptr, p->d_rec_ptr.ptr, p->d_rec_pidx.ptr, p->d_rec_w.ptr,
                                   p->d_rec_col.ptr, v, nr, p->d_pval.ptr, p->d_b.ptr, p->nrec_slot, ns,
                                   nc, s));
  HIP_OK(coarse_solve(p, p->d_b.ptr, lam_ptr(p), nullptr, s));
  HIP_OK(msfv::launch_prolong(p->d_prow.ptr, p->d_pcol.ptr, p->d_pval.ptr, p->d_t.ptr, P.ncv, ns, P.ncell,
                              p->d_fu.ptr, p->d_b.ptr, s));
  HIP_OK(msfv::launch_prolong(p->d_prow.ptr, p->d_pcol.ptr, p->d_pval.ptr, lam_ptr(p), P.ncv, ns, P.ncell,
                              p->d_fz.ptr, p->d_b.ptr, s));
  HIP_OK(msfv::launch_wfixed(p->g, P.ncell, ns, p->d_fu.ptr, p->d_fz.ptr, p->d_W.ptr, s));
  HIP_OK(msfv::launch_gfinal(p->d_sig.ptr, p->d_W.ptr, p->g, P.ncell, g_out, s));
  return MSFV_OK;
}

// Residual scratch of the allocation-free misfit entry point: the data D and
// the residual v = D - d_obs of one call (2 Nr Ns doubles), in a fixed
// device array instead of the problem's buffers.  Host code never passes the
// array's name to a kernel or a copy: it uses the device address returned by
// hipGetSymbolAddress, looked up once per device.
constexpr size_t kScratchDoubles = size_t(1) << 17;  // 1 MiB: Nr * Ns <= 65536
constexpr int kScratchDevices = 64;
static __device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_scratch_mu;
double* g_scratch_dev[kScratchDevices] = {};

// Device address of ``scratch`` on the current device.
msfv_status scratch_address(double** out) {
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kScratchDevices) return fail(MSFV_EDEVICE, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(MSFV_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_dev[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch_dev[dev];
  return MSFV_OK;
}

// J^T v and J dm of the problem's current model: adaptive basis (Sec. 4.3)
// or, with the basis frozen, the exact sensitivities of the fixed-basis
// model (eq. senssimple).
msfv_status jtv_model(msfv_problem* p, const double* v, double* g_out) {
  return p->frozen ? jtv_fixed_impl(p, v, g_out) : jtv_impl(p, v, g_out);
}

// Forward + J^T v with v given: one coarse launch for both sets of columns
// (a frozen basis takes its own J^T v, after the forward).
msfv_status forward_jtv_impl(msfv_problem* p, const double* m, const double* v, double* d_out,
                             double* g_out) {
  if (p->frozen) {
    msfv_status st = forward_impl(p, m, d_out, nullptr);
    return st == MSFV_OK ? jtv_fixed_impl(p, v, g_out) : st;
  }
  msfv_status st = fwd_begin(p, m);
  if (st == MSFV_OK) st = fwd_local(p);
  if (st == MSFV_OK) st = fwd_adj_coarse(p, v, d_out);
  if (st == MSFV_OK) st = adj_local(p);
  if (st == MSFV_OK) st = adj_end(p, g_out);
  return st;
}

msfv_status jvp_model(msfv_problem* p, const double* dm, double* dd_out) {
  return p->frozen ? jvp_fixed_impl(p, dm, dd_out) : jvp_impl(p, dm, dd_out);
}

}  // namespace

extern "C" {

const char* msfv_status_string(msfv_status s) {
  switch (s) {
    case MSFV_OK: return "ok";
    case MSFV_EINVAL: return "invalid argument";
    case MSFV_ENOMEM: return "out of memory";
    case MSFV_ENOCONV: return "iteration cap reached";
    case MSFV_ENONFINITE: return "non-finite model";
    case MSFV_EDEVICE: return "device error";
    case MSFV_ESTATE: return "call out of order";
  }
  return "unknown status";
}

const char* msfv_last_error(void) { return g_last_error.c_str(); }

msfv_status msfv_create(const msfv_config* cfg, void* hip_stream, msfv_problem** out) {
  if (!cfg || !out) return fail(MSFV_EINVAL, "null argument");
  *out = nullptr;
  msfv_problem* p = new (std::nothrow) msfv_problem();
  if (!p) return fail(MSFV_ENOMEM, "host allocation failed");
  p->cfg = *cfg;
  if (p->cfg.bc_mode != MSFV_BC_REDUCED && p->cfg.bc_mode != MSFV_BC_LAGRANGE) {
    delete p;
    return fail(MSFV_EINVAL, "bc_mode must be MSFV_BC_REDUCED or MSFV_BC_LAGRANGE");
  }
  if (p->cfg.local_rtol <= 0) p->cfg.local_rtol = 1e-13;
  if (p->cfg.local_maxit <= 0) p->cfg.local_maxit = 1000;
  if (p->cfg.coarse_rtol <= 0) p->cfg.coarse_rtol = 1e-13;
  if (p->cfg.coarse_maxit <= 0) p->cfg.coarse_maxit = 20000;
  if (p->cfg.coarse_precond != MSFV_COARSE_TWOLEVEL && p->cfg.coarse_precond != MSFV_COARSE_JACOBI &&
      p->cfg.coarse_precond != MSFV_COARSE_MULTI) {
    delete p;
    return fail(MSFV_EINVAL, "coarse_precond must be MSFV_COARSE_TWOLEVEL, _JACOBI or _MULTI");
  }
  p->stream = static_cast<hipStream_t>(hip_stream);
  std::string err = p->plan.build(cfg->dim, cfg->n, cfg->r);
  if (!err.empty()) {
    delete p;
    return fail(MSFV_EINVAL, err);
  }
  const msfv::Plan& P = p->plan;
  if (P.ncoarse > (1 << 21) || P.ncell >= (int64_t(1) << 31)) {
    delete p;
    return fail(MSFV_EINVAL, "more than 2^21 coarse vertices or 2^31 cells is not supported");
  }
  for (int k = 0; k < 3; ++k) p->g.n[k] = P.n[k];
  p->g.s1 = P.stride[1];
  p->g.s2 = P.stride[2];
  hipStream_t s = p->stream;
  auto cleanup = [&](msfv_status st) {
    delete p;
    return st;
  };
#define HIP_OR_CLEAN(expr)                                                                     \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess)                                                                      \
      return cleanup(fail(e_ == hipErrorOutOfMemory ? MSFV_ENOMEM : MSFV_EDEVICE,              \
                          std::string(#expr) + ": " + hipGetErrorString(e_)));                 \
  } while (0)
  HIP_OR_CLEAN(p->d_edges.upload(P.edges, s));
  for (const auto& E : P.edges) {
    const int k = (E.open_mask & 1) ? 0 : ((E.open_mask & 2) ? 1 : 2);
    p->edge_line = std::max(p->edge_line, E.cext[k]);
  }
  HIP_OR_CLEAN(p->d_faces.upload(P.faces, s));
  HIP_OR_CLEAN(p->d_blocks.upload(P.blocks, s));
  HIP_OR_CLEAN(p->d_prow.upload(P.prow, s));
  HIP_OR_CLEAN(p->d_pcol.upload(P.pcol, s));
  HIP_OR_CLEAN(p->d_krow.upload(P.krow, s));
  HIP_OR_CLEAN(p->d_kcol.upload(P.kcol, s));
  HIP_OR_CLEAN(p->d_kcptr.upload(P.kcptr, s));
  HIP_OR_CLEAN(p->d_kcidx.upload(P.kcidx, s));
  {
    // diagonal slots with the solver's padded row stride
    const int ldk = msfv::coarse_ldk(int(P.ncoarse));
    std::vector<int> slot(P.kdslot.size());
    for (size_t e = 0; e < slot.size(); ++e) {
      const int o = int(P.kdslot[e] / P.ncoarse), row = int(P.kdslot[e] % P.ncoarse);
      slot[e] = o * ldk + row;
    }
    HIP_OR_CLEAN(p->d_kdslot.upload(slot, s));
    HIP_OR_CLEAN(p->d_kdia.alloc(size_t(27) * ldk));
  }
  HIP_OR_CLEAN(hipMemsetAsync(p->d_kdia.ptr, 0, p->d_kdia.bytes(), s));
  if (p->cfg.coarse_precond == MSFV_COARSE_TWOLEVEL) {
    p->defl = msfv::coarse_is_large(P.ncv) ? msfv::coarse_defl_plan_large(P.ncv) : msfv::coarse_defl_plan(P.ncv);
    if (p->defl.ok) {
      HIP_OR_CLEAN(p->d_einv.alloc(size_t(p->defl.na) * p->defl.na));
      p->defl.einv = p->d_einv.ptr;
      HIP_OR_CLEAN(p->d_arows.upload(msfv::coarse_defl_rows(p->defl, P.ncv), s));
      p->defl.arows = p->d_arows.ptr;
    }
  }
  HIP_OR_CLEAN(p->d_pval.alloc(P.pcol.size()));
  HIP_OR_CLEAN(p->d_kval.alloc(std::max<size_t>(1, P.kcol.size())));
  HIP_OR_CLEAN(p->d_kent.alloc(std::max<int64_t>(1, P.kent_size)));
  HIP_OR_CLEAN(p->d_inbuf.alloc(std::max<int64_t>(1, P.inbuf_size)));
  HIP_OR_CLEAN(p->d_W.alloc(size_t(3) * P.ncell));
  {
    // full dual blocks: U^3 own cells, bounded by vertex planes on every axis
    auto full_of = [](const msfv::EntDesc& E) {
      const int U = E.uext[0];
      if ((U != 3 && U != 7) || E.uext[1] != U || E.uext[2] != U) return 0;
      if (E.open_mask != 7 || E.bounded_mask != 7 || E.nc != 8 || E.nu != U * U * U) return 0;
      for (int k = 0; k < 3; ++k)
        if (E.cext[k] != U + 2 || E.clo[k] != E.ulo[k] - 1) return 0;
      return U;
    };
    int best = 0, cnt3 = 0, cnt7 = 0;
    for (const auto& E : P.blocks) {
      const int u = P.dim == 3 ? full_of(E) : 0;
      cnt3 += u == 3;
      cnt7 += u == 7;
    }
    best = cnt7 >= cnt3 ? (cnt7 ? 7 : 0) : 3;
    std::vector<int> full, rest;
    for (int i = 0; i < int(P.blocks.size()); ++i)
      ((best && P.dim == 3 && full_of(P.blocks[i]) == best) ? full : rest).push_back(i);
    p->full_u = full.empty() ? 0 : best;
    p->nfull = int(full.size());
    p->nrest = int(rest.size());
    // launch order of the full blocks: dealt over the XCDs
    full = deal_over_xcds(full);
    full.insert(full.end(), rest.begin(), rest.end());
    p->h_blist = full;
    if (full.empty()) full.push_back(0);
    HIP_OR_CLEAN(p->d_blist.upload(full, s));
    // full faces (and the full dual blocks of a 2-D grid): U x U own cells
    // on a plane of axis k, bounded by vertex planes on both open axes (the
    // test the face kernels make to pick the body for the shape)
    auto face_of = [](const msfv::EntDesc& E, int* nax) {
      *nax = -1;
      if (E.nc != 4 || E.bounded_mask != E.open_mask) return 0;
      int U = 0;
      for (int k = 0; k < 3; ++k) {
        if ((E.open_mask >> k) & 1) {
          if (U == 0) U = E.uext[k];
          if (E.uext[k] != U || E.cext[k] != U + 2 || E.clo[k] != E.ulo[k] - 1) return 0;
        } else {
          if (*nax >= 0) return 0;
          *nax = k;
          if (E.uext[k] != 1 || E.cext[k] != 1 || E.clo[k] != E.ulo[k]) return 0;
        }
      }
      if (*nax < 0 || (U != 3 && U != 7) || E.nu != U * U) return 0;
      return U;
    };
    int fc3 = 0, fc7 = 0, nax = -1;
    for (const auto& E : P.faces) {
      const int u = face_of(E, &nax);
      fc3 += u == 3;
      fc7 += u == 7;
    }
    const int fbest = fc7 >= fc3 ? (fc7 ? 7 : 0) : 3;
    std::vector<int> by_axis[3], frest;
    for (int i = 0; i < int(P.faces.size()); ++i) {
      const int u = face_of(P.faces[i], &nax);
      (fbest && u == fbest ? by_axis[nax] : frest).push_back(i);
    }
    // launch order: the full faces of each plane axis, then the others, each
    // run dealt over the XCDs (the waves resident at a time mostly take one
    // body of the kernel)
    p->face_u = fbest;
    std::vector<int> faces;
    for (int k = 0; k < 3; ++k) {
      const std::vector<int> dealt = deal_over_xcds(by_axis[k]);
      faces.insert(faces.end(), dealt.begin(), dealt.end());
    }
    p->nface_full = int(faces.size());
    p->nface_rest = int(frest.size());
    p->faces_one_launch = P.caps_face.lane <= 64 && P.caps_face.col <= 1 && P.caps_face.nc <= 4;
    const std::vector<int> dealt = deal_over_xcds(frest);
    faces.insert(faces.end(), dealt.begin(), dealt.end());
    p->h_flist = faces;
    if (faces.empty()) faces.push_back(0);
    HIP_OR_CLEAN(p->d_flist.upload(faces, s));
  }
  {
    // scratch of the wave-level adjoint kernels (entities whose lane plane
    // and column fit one wavefront, and the full dual blocks, which always
    // take them): per entity 8 corners x the launch's own-cell cap
    auto fits = [](const msfv::Plan::Caps& c) { return c.lane <= 64 && c.col <= 7 && c.nc <= 8; };
    size_t mu = 0;
    if (fits(P.caps_block)) mu = std::max(mu, P.blocks.size() * 8 * size_t(std::max(1, P.max_nu_block)));
    if (p->nfull > 0) mu = std::max(mu, P.blocks.size() * 8 * size_t(p->full_u * p->full_u * p->full_u));
    if (fits(P.caps_face)) mu = std::max(mu, P.faces.size() * 8 * size_t(std::max(1, P.max_nu_face)));
    HIP_OR_CLEAN(p->d_mu.alloc(std::max<size_t>(1, mu)));
  }
  HIP_OR_CLEAN(p->d_m.alloc(P.ncell));
  HIP_OR_CLEAN(p->d_sig.alloc(P.ncell));
  HIP_OR_CLEAN(p->d_status.alloc(msfv::kStCount));
  HIP_OR_CLEAN(p->d_work.alloc(8));
  {
    const int nb = int(P.blocks.size()), nf = int(P.faces.size());
    const int cnt[4] = {nb, nb, nf, nf};
    for (int k = 0; k < 4; ++k) p->ent_off[k + 1] = p->ent_off[k] + cnt[k];
    HIP_OR_CLEAN(p->d_ent_it.alloc(std::max(1, p->ent_off[4])));
    HIP_OR_CLEAN(p->d_ent_res.alloc(size_t(8) * std::max(1, p->ent_off[4])));
    HIP_OR_CLEAN(p->d_ent_work.alloc(std::max(1, p->ent_off[4])));
    HIP_OR_CLEAN(hipMemsetAsync(p->d_ent_it.ptr, 0, p->d_ent_it.bytes(), s));
    HIP_OR_CLEAN(hipMemsetAsync(p->d_ent_res.ptr, 0, p->d_ent_res.bytes(), s));
    HIP_OR_CLEAN(hipMemsetAsync(p->d_ent_work.ptr, 0, p->d_ent_work.bytes(), s));
  }
  HIP_OR_CLEAN(hipMemsetAsync(p->d_work.ptr, 0, p->d_work.bytes(), s));
  HIP_OR_CLEAN(hipMemsetAsync(p->d_pval.ptr, 0, p->d_pval.bytes(), s));
  HIP_OR_CLEAN(hipMemsetAsync(p->d_inbuf.ptr, 0, p->d_inbuf.bytes(), s));
  HIP_OR_CLEAN(hipMemsetAsync(p->d_W.ptr, 0, p->d_W.bytes(), s));
  HIP_OR_CLEAN(hipMemsetAsync(p->d_status.ptr, 0, p->d_status.bytes(), s));
  std::vector<int> vrows;
  for (int K = 0; K < P.ncv[2]; ++K)
    for (int J = 0; J < P.ncv[1]; ++J)
      for (int I = 0; I < P.ncv[0]; ++I)
        vrows.push_back(P.prow[P.ax[0].v[I] + int64_t(P.ax[1].v[J]) * P.stride[1] +
                               int64_t(P.ax[2].v[K]) * P.stride[2]]);
  HIP_OR_CLEAN(p->d_vrows.upload(vrows, s));
  HIP_OR_CLEAN(msfv::launch_set_ones(p->d_vrows.ptr, int(vrows.size()), p->d_pval.ptr, s));
  HIP_OR_CLEAN(hipStreamSynchronize(s));
#undef HIP_OR_CLEAN
  *out = p;
  return MSFV_OK;
}

void msfv_destroy(msfv_problem* p) {
  if (!p) return;
  (void)hipStreamSynchronize(p->stream);
  delete p;
}

msfv_status msfv_set_sources(msfv_problem* p, int ns, const int* ptr, const int* cell, const double* val) {
  if (!p) return fail(MSFV_EINVAL, "null problem");
  Columns c;
  msfv_status st = check_columns(p, ns, ptr, cell, val, &c);
  if (st != MSFV_OK) return st;
  HIP_OK(hipStreamSynchronize(p->stream));
  p->src = std::move(c);
  p->electrodes_ready = false;
  p->have_forward = false;
  return MSFV_OK;
}

msfv_status msfv_set_receivers(msfv_problem* p, int nr, const int* ptr, const int* cell, const double* val) {
  if (!p) return fail(MSFV_EINVAL, "null problem");
  Columns c;
  msfv_status st = check_columns(p, nr, ptr, cell, val, &c);
  if (st != MSFV_OK) return st;
  HIP_OK(hipStreamSynchronize(p->stream));
  p->rec = std::move(c);
  p->electrodes_ready = false;
  p->have_forward = false;
  return MSFV_OK;
}

msfv_status msfv_forward(msfv_problem* p, const double* m, double* d_out, double* u_out) {
  if (!p || !m || !d_out) return fail(MSFV_EINVAL, "null argument");
  return forward_impl(p, m, d_out, u_out);
}

msfv_status msfv_jtv(msfv_problem* p, const double* v, double* g_out) {
  if (!p || !v || !g_out) return fail(MSFV_EINVAL, "null argument");
  return jtv_model(p, v, g_out);
}

msfv_status msfv_forward_jtv(msfv_problem* p, const double* m, const double* v, double* d_out,
                             double* g_out) {
  if (!p || !m || !v || !d_out || !g_out) return fail(MSFV_EINVAL, "null argument");
  return forward_jtv_impl(p, m, v, d_out, g_out);
}

msfv_status msfv_jvp(msfv_problem* p, const double* dm, double* dd_out) {
  if (!p || !dm || !dd_out) return fail(MSFV_EINVAL, "null argument");
  return jvp_model(p, dm, dd_out);
}

msfv_status msfv_set_basis(msfv_problem* p, int mode) {
  if (!p) return fail(MSFV_EINVAL, "null problem");
  if (mode != MSFV_BASIS_ADAPTIVE && mode != MSFV_BASIS_FROZEN)
    return fail(MSFV_EINVAL, "mode must be MSFV_BASIS_ADAPTIVE or MSFV_BASIS_FROZEN");
  if (mode == MSFV_BASIS_ADAPTIVE) {
    p->frozen = false;
    return MSFV_OK;
  }
  if (!p->basis_ready) return fail(MSFV_ESTATE, "freezing the basis needs a forward first");
  HIP_OK(hipStreamSynchronize(p->stream));
  // the fixed-basis sensitivities' workspace, now rather than inside a
  // later call (which may be captured in a graph)
  msfv_status st = fine_ready(p);
  if (st == MSFV_OK) st = sens_ready_alloc(p);
  if (st != MSFV_OK) return st;
  HIP_OK(hipStreamSynchronize(p->stream));
  p->frozen = true;
  return MSFV_OK;
}

msfv_status msfv_jvp_fixed(msfv_problem* p, const double* dm, double* dd_out) {
  if (!p || !dm || !dd_out) return fail(MSFV_EINVAL, "null argument");
  return jvp_fixed_impl(p, dm, dd_out);
}

msfv_status msfv_jtv_fixed(msfv_problem* p, const double* v, double* g_out) {
  if (!p || !v || !g_out) return fail(MSFV_EINVAL, "null argument");
  return jtv_fixed_impl(p, v, g_out);
}

msfv_status msfv_misfit_grad(msfv_problem* p, const double* m, const double* d_obs, double* phi_out,
                             double* g_out) {
  if (!p || !m || !d_obs || !phi_out || !g_out) return fail(MSFV_EINVAL, "null argument");
  msfv_status st = ensure_ready(p);
  if (st != MSFV_OK) return st;
  st = forward_impl(p, m, p->d_D.ptr, nullptr);
  if (st != MSFV_OK) return st;
  const long long n = (long long)p->rec.count * p->src.count;
  STAGE(MSFV_STAGE_RESIDUAL, msfv::launch_residual(p->d_D.ptr, d_obs, p->d_v.ptr, n, phi_out, p->stream));
  return jtv_model(p, p->d_v.ptr, g_out);
}

msfv_status msfv_misfit_grad_noalloc(msfv_problem* p, const double* m, const double* d_obs,
                                     double* phi_out, double* g_out) {
  if (!p || !m || !d_obs || !phi_out || !g_out) return fail(MSFV_EINVAL, "null argument");
  const long long n = (long long)p->rec.count * p->src.count;
  if (2 * n > (long long)kScratchDoubles)
    return fail(MSFV_EINVAL, "msfv_misfit_grad_noalloc: Nr * Ns = " + std::to_string(n) +
                                 " exceeds the scratch maximum of " + std::to_string(kScratchDoubles / 2));
  if (p->src.count <= 0 || p->rec.count <= 0) return fail(MSFV_ESTATE, "no sources or receivers set");
  // the electrode tables and coarse vectors are (re)allocated by the first
  // forward after the sources or receivers change; this entry point does not
  if (!p->electrodes_ready)
    return fail(MSFV_ESTATE, "msfv_misfit_grad_noalloc: run msfv_forward or msfv_misfit_grad once after "
                             "setting the sources and receivers");
  double* sc = nullptr;
  msfv_status st = scratch_address(&sc);
  if (st != MSFV_OK) return st;
  double* D = sc;
  double* v = sc + n;
  const bool prof = p->prof.on;  // stage events may create HIP events: off for this call
  p->prof.on = false;
  st = forward_impl(p, m, D, nullptr);
  if (st == MSFV_OK) {
    const hipError_t e = msfv::launch_residual(D, d_obs, v, n, phi_out, p->stream);
    st = e == hipSuccess ? MSFV_OK : fail(MSFV_EDEVICE, std::string("launch_residual: ") + hipGetErrorString(e));
  }
  if (st == MSFV_OK) st = jtv_model(p, v, g_out);
  p->prof.on = prof;
  return st;
}

namespace {
// Status words of the last call (the caller has synchronised).
msfv_status check_status(msfv_problem* p) {
  int st[msfv::kStCount];
  HIP_OK(hipMemcpy(st, p->d_status.ptr, sizeof st, hipMemcpyDeviceToHost));
  if (st[msfv::kStNonfinite]) return fail(MSFV_ENONFINITE, "m contains NaN or Inf");
  if (st[msfv::kStLocalNoconv] || st[msfv::kStCoarseNoconv])
    return fail(MSFV_ENOCONV, "an iteration reached its cap");
  return MSFV_OK;
}
}  // namespace

msfv_status msfv_sync(msfv_problem* p) {
  if (!p) return fail(MSFV_EINVAL, "null problem");
  HIP_OK(hipStreamSynchronize(p->stream));
  return check_status(p);
}

msfv_status msfv_get_sizes(msfv_problem* p, msfv_sizes* out) {
  if (!p || !out) return fail(MSFV_EINVAL, "null argument");
  const msfv::Plan& P = p->plan;
  out->ncell = P.ncell;
  out->ncoarse = P.ncoarse;
  out->nnz_p = (long long)P.pcol.size();
  out->nnz_k = (long long)P.kcol.size();
  out->nsrc = p->src.count;
  out->nrec = p->rec.count;
  out->nblock = int(P.blocks.size());
  out->nface = P.dim == 3 ? int(P.faces.size()) : 0;
  out->nedge = int(P.edges.size());
  out->workspace_bytes = (long long)p->workspace_bytes();
  out->pairs_block = out->pairs_face = 0;
  for (const auto& E : P.blocks) out->pairs_block += (long long)E.nc * E.nu;
  for (const auto& E : P.faces) out->pairs_face += (long long)E.nc * E.nu;
  return MSFV_OK;
}

msfv_status msfv_get_prolongation(msfv_problem* p, int* row_ptr, int* col, double* val) {
  if (!p) return fail(MSFV_EINVAL, "null problem");
  HIP_OK(hipStreamSynchronize(p->stream));
  const msfv::Plan& P = p->plan;
  if (row_ptr) std::memcpy(row_ptr, P.prow.data(), P.prow.size() * sizeof(int));
  if (col) std::memcpy(col, P.pcol.data(), P.pcol.size() * sizeof(int));
  if (val) HIP_OK(hipMemcpy(val, p->d_pval.ptr, P.pcol.size() * sizeof(double), hipMemcpyDeviceToHost));
  return MSFV_OK;
}

msfv_status msfv_get_coarse(msfv_problem* p, int* row_ptr, int* col, double* val, double* t_out) {
  if (!p) return fail(MSFV_EINVAL, "null problem");
  HIP_OK(hipStreamSynchronize(p->stream));
  const msfv::Plan& P = p->plan;
  if (row_ptr) std::memcpy(row_ptr, P.krow.data(), P.krow.size() * sizeof(int));
  if (col) std::memcpy(col, P.kcol.data(), P.kcol.size() * sizeof(int));
  if (val) HIP_OK(hipMemcpy(val, p->d_kval.ptr, P.kcol.size() * sizeof(double), hipMemcpyDeviceToHost));
  if (t_out && p->d_t.ptr)
    HIP_OK(hipMemcpy(t_out, p->d_t.ptr, size_t(P.ncoarse) * p->src.count * sizeof(double),
                     hipMemcpyDeviceToHost));
  return MSFV_OK;
}

msfv_status msfv_profile_enable(msfv_problem* p, int enable) {
  if (!p) return fail(MSFV_EINVAL, "null problem");
  HIP_OK(hipStreamSynchronize(p->stream));
  p->prof.on = enable != 0;
  p->prof.recs.clear();
  p->prof.next = 0;
  HIP_OK(hipMemset(p->d_work.ptr, 0, p->d_work.bytes()));
  HIP_OK(hipMemset(p->d_ent_work.ptr, 0, p->d_ent_work.bytes()));
  return MSFV_OK;
}

msfv_status msfv_profile_read(msfv_problem* p, msfv_profile* out) {
  if (!p || !out) return fail(MSFV_EINVAL, "null argument");
  HIP_OK(hipStreamSynchronize(p->stream));
  std::memset(out, 0, sizeof *out);
  for (auto& r : p->prof.recs) {
    float ms = 0.f;
    HIP_OK(hipEventElapsedTime(&ms, std::get<1>(r), std::get<2>(r)));
    const int id = std::get<0>(r);
    if (id >= 0 && id < MSFV_NSTAGE) {
      out->ms[id] += ms;
      out->count[id] += 1;
    }
  }
  p->prof.recs.clear();
  p->prof.next = 0;
  HIP_OK(hipMemcpy(out->work, p->d_work.ptr, sizeof out->work, hipMemcpyDeviceToHost));
  HIP_OK(hipMemset(p->d_work.ptr, 0, p->d_work.bytes()));
  // local stages: per-entity cell-iterations, summed here in entity order
  std::vector<unsigned long long> ew(p->d_ent_work.n);
  if (!ew.empty())
    HIP_OK(hipMemcpy(ew.data(), p->d_ent_work.ptr, p->d_ent_work.bytes(), hipMemcpyDeviceToHost));
  for (int slot = 0; slot < 4; ++slot) {
    unsigned long long t = 0;
    for (int e = p->ent_off[slot]; e < p->ent_off[slot + 1]; ++e) t += ew[e];
    out->work[slot] = t;
  }
  HIP_OK(hipMemset(p->d_ent_work.ptr, 0, p->d_ent_work.bytes()));
  return MSFV_OK;
}

const char* msfv_stage_name(int stage) {
  static const char* names[MSFV_NSTAGE] = {
      "copy_m", "check_finite", "edge_fwd", "face_fwd", "block_fwd", "kassemble", "coarse_rhs",
      "coarse_fwd", "data", "prolong", "adj_rhs", "coarse_adj", "sload", "block_adj",
      "face_adj", "edge_adj", "gfinal", "residual", "coarse_setup"};
  if (stage < 0 || stage >= MSFV_NSTAGE) return "unknown";
  return names[stage];
}

msfv_status msfv_get_stats(msfv_problem* p, msfv_stats* out) {
  if (!p || !out) return fail(MSFV_EINVAL, "null argument");
  HIP_OK(hipStreamSynchronize(p->stream));
  int st[msfv::kStCount];
  HIP_OK(hipMemcpy(st, p->d_status.ptr, sizeof st, hipMemcpyDeviceToHost));
  std::vector<int> it(p->d_ent_it.n);
  if (!it.empty())
    HIP_OK(hipMemcpy(it.data(), p->d_ent_it.ptr, p->d_ent_it.bytes(), hipMemcpyDeviceToHost));
  int itmax = 0;
  for (int v : it) itmax = std::max(itmax, v);
  out->local_max_it = itmax;
  out->local_noconv = st[msfv::kStLocalNoconv];
  out->coarse_max_it = st[msfv::kStCoarseMaxIt];
  out->coarse_noconv = st[msfv::kStCoarseNoconv];
  out->nonfinite = st[msfv::kStNonfinite];
  auto res = [&](int slot) {
    unsigned long long bits;
    std::memcpy(&bits, st + slot, sizeof bits);
    double v;
    std::memcpy(&v, &bits, sizeof v);
    return std::sqrt(v);
  };
  std::vector<double> lr(p->d_ent_res.n);
  if (!lr.empty())
    HIP_OK(hipMemcpy(lr.data(), p->d_ent_res.ptr, p->d_ent_res.bytes(), hipMemcpyDeviceToHost));
  double lmax = 0.0;
  for (double v : lr) lmax = (v >= 0.0) ? std::max(lmax, v) : HUGE_VAL;  // a NaN counts as +inf
  out->local_max_res = std::sqrt(lmax);
  out->coarse_max_res = res(msfv::kStCoarseRes);
  return MSFV_OK;
}


// ---- batches ----------------------------------------------------------------

struct msfv_batch {
  std::vector<msfv_problem*> probs;
  std::vector<int> order;        // issue order: most fine cells first
  hipStream_t main = nullptr;    // caller's stream
  std::vector<hipStream_t> pool; // owned, default priority
  std::vector<hipEvent_t> done;  // one per pool stream
  hipEvent_t fork = nullptr;
  int streams = 8;
  bool graphs = true;
  struct Graph {
    const double* m = nullptr;
    const double* v = nullptr;
    double* d = nullptr;
    double* g = nullptr;
    unsigned long long generation = ~0ull;
    hipGraphExec_t exec = nullptr;
  };
  std::vector<Graph> cache;      // one per problem
  // shared mode: the local solves of the problems run as shared launches,
  // one per kernel class and stage, over (problem, entity) items.  The
  // problems are split into `shared` pipelines, each issued by a host thread
  // of its own on its own streams, so one pipeline's local launches overlap
  // another's coarse solves.
  int shared = 0;
  struct Group {
    int stage = 0;   // 1 edges, 2 faces (2-D blocks), 3 dual blocks
    bool adj = false;
    int klass = 0;   // kernel class of the local solves (edges: 0)
    msfv::LocalParams caps;  // largest caps of the class, for the launch
    std::vector<int2> items;
    DevBuf<int2> d_items;
  };
  struct Pipeline {
    std::vector<int> members;                  // problem indices, largest first
    std::vector<std::unique_ptr<Group>> groups;
    DevBuf<msfv::LocalParams> d_params;
    std::vector<unsigned long long> gen;       // member generations the groups were built for
    hipStream_t main = nullptr;                // shared launches
    std::vector<hipStream_t> streams;          // per-problem parts
    hipEvent_t fork = nullptr, fin = nullptr;
    std::vector<hipEvent_t> done;
    ~Pipeline() {
      if (fork) (void)hipEventDestroy(fork);
      if (fin) (void)hipEventDestroy(fin);
      for (auto e : done) (void)hipEventDestroy(e);
    }
  };
  std::vector<std::unique_ptr<Pipeline>> pipes;
  int pipes_streams = 0;  // stream count the pipelines were laid out for
  ~msfv_batch() {
    if (main) (void)hipStreamSynchronize(main);
    for (auto s : pool) (void)hipStreamSynchronize(s);
    for (auto& c : cache)
      if (c.exec) (void)hipGraphExecDestroy(c.exec);
    for (auto e : done) (void)hipEventDestroy(e);
    if (fork) (void)hipEventDestroy(fork);
    for (auto s : pool) (void)hipStreamDestroy(s);
  }
};

namespace {

// forward + J^T v of one problem on stream s (eager or through its graph)
msfv_status batch_one(msfv_batch* b, int i, const double* m, const double* v, double* d, double* g,
                      hipStream_t s) {
  msfv_problem* p = b->probs[i];
  const hipStream_t own = p->stream;
  const bool prof = p->prof.on;
  p->stream = s;
  p->prof.on = false;
  msfv_status st = MSFV_OK;
  // the large coarse solver polls from the host, which a graph cannot hold
  if (!b->graphs || coarse_multi(p)) {
    st = forward_jtv_impl(p, m, v, d, g);
  } else {
    msfv_batch::Graph& c = b->cache[i];
    if (!c.exec || c.m != m || c.v != v || c.d != d || c.g != g || c.generation != p->generation) {
      if (c.exec) (void)hipGraphExecDestroy(c.exec);
      c.exec = nullptr;
      hipGraph_t graph = nullptr;
      hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) {
        st = forward_jtv_impl(p, m, v, d, g);
        e = hipStreamEndCapture(s, &graph);
        if (st == MSFV_OK && e == hipSuccess) e = hipGraphInstantiate(&c.exec, graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
      }
      if (st == MSFV_OK && e != hipSuccess) st = fail(MSFV_EDEVICE, hipGetErrorString(e));
      if (st == MSFV_OK) {
        c.m = m;
        c.v = v;
        c.d = d;
        c.g = g;
        c.generation = p->generation;
      }
    }
    if (st == MSFV_OK) {
      hipError_t e = hipGraphLaunch(c.exec, s);
      if (e != hipSuccess) st = fail(MSFV_EDEVICE, hipGetErrorString(e));
    }
  }
  p->stream = own;
  p->prof.on = prof;
  return st;
}

// The shared launches of a pipeline: per member problem, stage and kernel
// class one parameter block; items grouped by (stage, direction, class).
msfv_status shared_build(msfv_batch* b, msfv_batch::Pipeline* pl) {
  std::vector<msfv::LocalParams> params;
  std::map<std::tuple<int, int, int>, msfv_batch::Group*> index;
  pl->groups.clear();
  auto group = [&](int stage, bool adj, int klass) {
    auto key = std::make_tuple(stage, adj ? 1 : 0, klass);
    auto it = index.find(key);
    if (it != index.end()) return it->second;
    pl->groups.emplace_back(new msfv_batch::Group());
    msfv_batch::Group* g = pl->groups.back().get();
    g->stage = stage;
    g->adj = adj;
    g->klass = klass;
    index[key] = g;
    return g;
  };
  auto add = [&](msfv::LocalParams lp, int stage, bool adj, int klass, const int* ids, int count) {
    if (count <= 0) return MSFV_OK;
    if (stage > 1 && klass == msfv::kClassNone) return fail(MSFV_EINVAL, "an entity does not fit any local kernel");
    lp.ent_work = nullptr;
    lp.ent_list = nullptr;
    if (stage > 1) lp.uni_cap = msfv::local_class_uni_cap(lp, klass);
    const int pid = int(params.size());
    params.push_back(lp);
    msfv_batch::Group* g = group(stage, adj, klass);
    msfv::LocalParams& c = g->caps;
    c.nu_cap = std::max(c.nu_cap, lp.nu_cap);
    c.sig_cap = std::max(c.sig_cap, lp.sig_cap);
    c.lane_cap = std::max(c.lane_cap, lp.lane_cap);
    c.col_cap = std::max(c.col_cap, lp.col_cap);
    c.nc_cap = std::max(c.nc_cap, lp.nc_cap);
    c.plane_cap = std::max(c.plane_cap, lp.plane_cap);
    c.line_cap = std::max(c.line_cap, lp.line_cap);
    for (int k = 0; k < count; ++k) g->items.push_back(make_int2(pid, ids ? ids[k] : k));
    return MSFV_OK;
  };
  for (int i : pl->members) {
    msfv_problem* p = b->probs[i];
    const msfv::Plan& P = p->plan;
    for (int dir = 0; dir < 2; ++dir) {
      const bool adj = dir == 1;
      msfv_status st = add(local_params(p, 1, adj), 1, adj, 0, nullptr, int(P.edges.size()));
      if (st != MSFV_OK) return st;
      msfv::LocalParams lf = local_params(p, 2, adj);
      if (p->nface_full > 0 && p->faces_one_launch) {
        st = add(lf, 2, adj, msfv::faces_class(p->face_u), p->h_flist.data(), p->nface_full + p->nface_rest);
      } else {
        if (p->nface_full > 0) {
          msfv::LocalParams lff = lf;
          face_caps(lff, p->face_u);
          st = add(lff, 2, adj, msfv::faces_class(p->face_u), p->h_flist.data(), p->nface_full);
        }
        if (st == MSFV_OK)
          st = add(lf, 2, adj, msfv::local_class(lf), p->h_flist.data() + p->nface_full, p->nface_rest);
      }
      if (st != MSFV_OK) return st;
      if (P.dim == 3) {
        msfv::LocalParams lb = local_params(p, 3, adj);
        if (p->nfull > 0) {
          msfv::LocalParams lfull = lb;
          full_caps(lfull, p->full_u);
          st = add(lfull, 3, adj, msfv::full_class(p->full_u), p->h_blist.data(), p->nfull);
        }
        if (st == MSFV_OK)
          st = add(lb, 3, adj, msfv::local_class(lb), p->h_blist.data() + p->nfull, p->nrest);
        if (st != MSFV_OK) return st;
      }
    }
  }
  hipStream_t s = pl->main;
  HIP_OK(pl->d_params.upload(params, s));
  for (auto& g : pl->groups) {
    HIP_OK(g->d_items.upload(g->items, s));
    g->caps.multi = pl->d_params.ptr;
    g->caps.items = g->d_items.ptr;
    g->caps.nent = int(g->items.size());
  }
  // launch order: forward edges, faces, blocks; adjoint blocks, faces, edges
  std::stable_sort(pl->groups.begin(), pl->groups.end(), [](const auto& x, const auto& y) {
    const int kx = x->adj ? 10 - x->stage : x->stage, ky = y->adj ? 10 - y->stage : y->stage;
    return kx < ky;
  });
  pl->gen.clear();
  for (int i : pl->members) pl->gen.push_back(b->probs[i]->generation);
  return MSFV_OK;
}

// Issue fn(problem, index) for every member of a pipeline over its streams
// (forked from and joined into its main stream), members on the host-polled
// coarse solver from worker threads.
extern "C++" template <typename Fn>
msfv_status issue_each(msfv_batch* b, msfv_batch::Pipeline* pl, Fn fn) {
  const int ns = int(pl->streams.size());
  HIP_OK(hipEventRecord(pl->fork, pl->main));
  for (int k = 0; k < ns; ++k) HIP_OK(hipStreamWaitEvent(pl->streams[k], pl->fork, 0));
  std::vector<int> polled, plain;
  for (int i : pl->members) (ns > 1 && coarse_multi(b->probs[i]) ? polled : plain).push_back(i);
  const int nw = polled.empty() ? 0 : std::min<int>(int(polled.size()), std::max(1, ns / 2));
  std::vector<msfv_status> wst(nw, MSFV_OK);
  std::vector<std::string> werr(nw);
  std::vector<std::thread> workers;
  int device = 0;
  if (nw > 0) HIP_OK(hipGetDevice(&device));
  auto one = [&](int i, hipStream_t s) {
    msfv_problem* p = b->probs[i];
    const hipStream_t own = p->stream;
    const bool prof = p->prof.on;
    p->stream = s;
    p->prof.on = false;
    const msfv_status st = fn(p, i);
    p->stream = own;
    p->prof.on = prof;
    return st;
  };
  for (int w = 0; w < nw; ++w)
    workers.emplace_back([&, w]() {
      (void)hipSetDevice(device);
      for (size_t k = w; k < polled.size(); k += nw) {
        const msfv_status st = one(polled[k], pl->streams[w]);
        if (st != MSFV_OK) {
          wst[w] = st;
          werr[w] = msfv_last_error();
          return;
        }
      }
    });
  msfv_status st = MSFV_OK;
  const int nplain = ns - nw;
  for (size_t k = 0; k < plain.size() && st == MSFV_OK; ++k)
    st = one(plain[k], nplain > 0 ? pl->streams[nw + int(k % nplain)] : pl->main);
  for (auto& t : workers) t.join();
  if (st != MSFV_OK) return st;
  for (int w = 0; w < nw; ++w)
    if (wst[w] != MSFV_OK) return fail(wst[w], werr[w]);
  for (int k = 0; k < ns; ++k) {
    HIP_OK(hipEventRecord(pl->done[k], pl->streams[k]));
    HIP_OK(hipStreamWaitEvent(pl->main, pl->done[k], 0));
  }
  return MSFV_OK;
}

// One pipeline: per-problem parts on its streams, the local solves of its
// members in shared launches on its main stream.
msfv_status pipeline_run(msfv_batch* b, msfv_batch::Pipeline* pl, const double* const* m,
                         const double* const* v, double* const* d_out, double* const* g_out) {
  bool rebuild = pl->groups.empty() || pl->gen.size() != pl->members.size();
  for (size_t k = 0; !rebuild && k < pl->members.size(); ++k)
    rebuild = pl->gen[k] != b->probs[pl->members[k]]->generation;
  if (rebuild) {
    msfv_status st = shared_build(b, pl);
    if (st != MSFV_OK) return st;
  }
  msfv_status st = issue_each(b, pl, [&](msfv_problem* p, int i) { return fwd_begin(p, m[i]); });
  if (st != MSFV_OK) return st;
  for (auto& g : pl->groups)
    if (!g->adj)
      HIP_OK(g->stage == 1 ? msfv::launch_edge_multi(g->caps, false, pl->main)
                           : msfv::launch_local_multi(g->caps, g->klass, false, pl->main));
  st = issue_each(b, pl, [&](msfv_problem* p, int i) { return fwd_adj_coarse(p, v[i], d_out[i]); });
  if (st != MSFV_OK) return st;
  for (auto& g : pl->groups)
    if (g->adj)
      HIP_OK(g->stage == 1 ? msfv::launch_edge_multi(g->caps, true, pl->main)
                           : msfv::launch_local_multi(g->caps, g->klass, true, pl->main));
  return issue_each(b, pl, [&](msfv_problem* p, int i) { return adj_end(p, g_out[i]); });
}

// Lay the problems out over b->shared pipelines: members dealt round-robin
// from the largest-first order; pipeline q gets pool stream q as its main
// stream and the pool streams k >= pipes (k < streams) with k % pipes == q.
msfv_status shared_layout(msfv_batch* b) {
  const int np = std::max(1, std::min<int>(b->shared, int(b->probs.size())));
  const int ns = std::max(b->streams, np);
  if (int(b->pipes.size()) == np && b->pipes_streams == ns) return MSFV_OK;
  b->pipes.clear();
  for (int q = 0; q < np; ++q) {
    std::unique_ptr<msfv_batch::Pipeline> pl(new msfv_batch::Pipeline());
    for (int k = q; k < int(b->order.size()); k += np) pl->members.push_back(b->order[k]);
    pl->main = b->pool[q];
    for (int k = np; k < ns && k < int(b->pool.size()); ++k)
      if (k % np == q) pl->streams.push_back(b->pool[k]);
    HIP_OK(hipEventCreateWithFlags(&pl->fork, hipEventDisableTiming));
    HIP_OK(hipEventCreateWithFlags(&pl->fin, hipEventDisableTiming));
    for (size_t k = 0; k < pl->streams.size(); ++k) {
      hipEvent_t e = nullptr;
      HIP_OK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      pl->done.push_back(e);
    }
    b->pipes.push_back(std::move(pl));
  }
  b->pipes_streams = ns;
  return MSFV_OK;
}

// Shared mode: the pipelines run concurrently, each issued by a host thread.
msfv_status shared_run(msfv_batch* b, const double* const* m, const double* const* v,
                       double* const* d_out, double* const* g_out) {
  msfv_status st = shared_layout(b);
  if (st != MSFV_OK) return st;
  HIP_OK(hipEventRecord(b->fork, b->main));
  for (auto& pl : b->pipes) HIP_OK(hipStreamWaitEvent(pl->main, b->fork, 0));
  const int np = int(b->pipes.size());
  std::vector<msfv_status> pst(np, MSFV_OK);
  std::vector<std::string> perr(np);
  if (np == 1) {
    pst[0] = pipeline_run(b, b->pipes[0].get(), m, v, d_out, g_out);
    if (pst[0] != MSFV_OK) perr[0] = msfv_last_error();
  } else {
    int device = 0;
    HIP_OK(hipGetDevice(&device));
    std::vector<std::thread> th;
    for (int q = 0; q < np; ++q)
      th.emplace_back([&, q]() {
        (void)hipSetDevice(device);
        pst[q] = pipeline_run(b, b->pipes[q].get(), m, v, d_out, g_out);
        if (pst[q] != MSFV_OK) perr[q] = msfv_last_error();
      });
    for (auto& t : th) t.join();
  }
  for (int q = 0; q < np; ++q)
    if (pst[q] != MSFV_OK) return fail(pst[q], perr[q]);
  for (auto& pl : b->pipes) {
    HIP_OK(hipEventRecord(pl->fin, pl->main));
    HIP_OK(hipStreamWaitEvent(b->main, pl->fin, 0));
  }
  return MSFV_OK;
}

msfv_status batch_run(msfv_batch* b, const double* const* m, const double* const* v,
                      double* const* d_out, double* const* g_out) {
  const int n = int(b->probs.size());
  bool any_frozen = false;
  for (int i = 0; i < n; ++i) {
    if (!m[i] || !v[i] || !d_out[i] || !g_out[i]) return fail(MSFV_EINVAL, "null buffer in batch");
    msfv_status st = ensure_ready(b->probs[i]);
    if (st != MSFV_OK) return st;
    any_frozen |= b->probs[i]->frozen;
  }
  // frozen bases keep their own path (no local solves to share)
  if (b->shared > 0 && !any_frozen) return shared_run(b, m, v, d_out, g_out);
  const int ns = std::min<int>(b->streams, int(b->pool.size()));
  HIP_OK(hipEventRecord(b->fork, b->main));
  for (int k = 0; k < ns; ++k) HIP_OK(hipStreamWaitEvent(b->pool[k], b->fork, 0));
  // Problems on the multi-launch coarse solver poll its stop flags from the
  // host, which would hold up the issue of every other problem.  With more
  // than one stream they get streams of their own, each driven by a host
  // thread; the other problems are issued round-robin on the remaining
  // streams by this thread.  Either list keeps the largest-first order.
  std::vector<int> polled, plain;
  for (int q = 0; q < n; ++q) {
    const int i = b->order[q];
    (ns > 1 && coarse_multi(b->probs[i]) ? polled : plain).push_back(i);
  }
  const int nw = polled.empty() ? 0 : std::min<int>(int(polled.size()), std::max(1, ns / 2));
  std::vector<msfv_status> wst(nw, MSFV_OK);
  std::vector<std::string> werr(nw);
  std::vector<std::thread> workers;
  int device = 0;
  if (nw > 0) HIP_OK(hipGetDevice(&device));
  for (int w = 0; w < nw; ++w)
    workers.emplace_back([&, w]() {
      (void)hipSetDevice(device);  // the caller's device, current in this thread too
      for (size_t k = w; k < polled.size(); k += nw) {
        const int i = polled[k];
        const msfv_status st = batch_one(b, i, m[i], v[i], d_out[i], g_out[i], b->pool[w]);
        if (st != MSFV_OK) {
          wst[w] = st;
          werr[w] = msfv_last_error();
          return;
        }
      }
    });
  msfv_status st = MSFV_OK;
  const int nplain = ns - nw;
  for (size_t k = 0; k < plain.size() && st == MSFV_OK; ++k) {
    const int i = plain[k];
    st = batch_one(b, i, m[i], v[i], d_out[i], g_out[i], b->pool[nw + int(k % nplain)]);
  }
  for (auto& t : workers) t.join();
  if (st != MSFV_OK) return st;
  for (int w = 0; w < nw; ++w)
    if (wst[w] != MSFV_OK) return fail(wst[w], werr[w]);
  for (int k = 0; k < ns; ++k) {
    HIP_OK(hipEventRecord(b->done[k], b->pool[k]));
    HIP_OK(hipStreamWaitEvent(b->main, b->done[k], 0));
  }
  return MSFV_OK;
}

}  // namespace

msfv_status msfv_batch_create(int count, msfv_problem* const* problems, void* hip_stream,
                              msfv_batch** out) {
  if (!out || !problems || count <= 0) return fail(MSFV_EINVAL, "bad batch arguments");
  *out = nullptr;
  std::unique_ptr<msfv_batch> b(new msfv_batch());
  for (int i = 0; i < count; ++i) {
    if (!problems[i]) return fail(MSFV_EINVAL, "null problem in batch");
    for (int j = 0; j < i; ++j)
      if (problems[j] == problems[i]) return fail(MSFV_EINVAL, "a problem appears twice in the batch");
    b->probs.push_back(problems[i]);
  }
  b->order.resize(count);
  for (int i = 0; i < count; ++i) b->order[i] = i;
  std::stable_sort(b->order.begin(), b->order.end(), [&](int x, int y) {
    return b->probs[x]->plan.ncell > b->probs[y]->plan.ncell;
  });
  b->cache.resize(count);
  b->main = static_cast<hipStream_t>(hip_stream);
  constexpr int kPool = 16;
  for (int k = 0; k < kPool; ++k) {
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess)
      return fail(MSFV_EDEVICE, "hipStreamCreate failed");
    b->pool.push_back(s);
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
      return fail(MSFV_EDEVICE, "hipEventCreate failed");
    b->done.push_back(e);
  }
  if (hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess)
    return fail(MSFV_EDEVICE, "hipEventCreate failed");
  b->streams = std::min(8, count);
  *out = b.release();
  return MSFV_OK;
}

void msfv_batch_destroy(msfv_batch* b) { delete b; }

msfv_status msfv_batch_forward_jtv(msfv_batch* b, const double* const* m, const double* const* v,
                                   double* const* d_out, double* const* g_out) {
  if (!b || !m || !v || !d_out || !g_out) return fail(MSFV_EINVAL, "null argument");
  return batch_run(b, m, v, d_out, g_out);
}

msfv_status msfv_batch_sync(msfv_batch* b) {
  if (!b) return fail(MSFV_EINVAL, "null batch");
  HIP_OK(hipStreamSynchronize(b->main));
  for (auto s : b->pool) HIP_OK(hipStreamSynchronize(s));
  for (msfv_problem* p : b->probs) {
    msfv_status st = check_status(p);
    if (st != MSFV_OK) return st;
  }
  return MSFV_OK;
}

msfv_status msfv_batch_set_options(msfv_batch* b, int streams, int graphs, int shared) {
  if (!b) return fail(MSFV_EINVAL, "null batch");
  if (streams < 1 || streams > int(b->pool.size())) return fail(MSFV_EINVAL, "streams outside [1, 16]");
  if (shared < 0 || shared > 8) return fail(MSFV_EINVAL, "shared (pipelines) outside [0, 8]");
  HIP_OK(hipStreamSynchronize(b->main));
  for (auto s : b->pool) HIP_OK(hipStreamSynchronize(s));
  b->streams = streams;
  b->graphs = graphs != 0;
  b->shared = shared;
  return MSFV_OK;
}

msfv_status msfv_batch_get_options(msfv_batch* b, int* streams, int* graphs, int* shared) {
  if (!b) return fail(MSFV_EINVAL, "null batch");
  if (streams) *streams = b->streams;
  if (graphs) *graphs = b->graphs ? 1 : 0;
  if (shared) *shared = b->shared;
  return MSFV_OK;
}

msfv_status msfv_batch_autotune(msfv_batch* b, const double* const* m, const double* const* v,
                                double* const* d_out, double* const* g_out, int* streams_out,
                                int* graphs_out, int* shared_out) {
  if (!b || !m || !v || !d_out || !g_out) return fail(MSFV_EINVAL, "null argument");
  const int count = int(b->probs.size());
  double best = 1e300;
  int best_s = b->streams, best_sh = b->shared;
  bool best_g = b->graphs;
  // candidates: shared launches of the local solves in 1, 2, 4 or 8
  // pipelines, or each problem's whole sequence on the stream pool, replayed
  // from HIP graphs or issued eagerly; each over 1..16 streams
  struct Cand {
    int shared;
    bool graphs;
  };
  for (const Cand c : {Cand{1, false}, Cand{2, false}, Cand{4, false}, Cand{8, false}, Cand{0, true},
                       Cand{0, false}}) {
    if (c.shared > count) continue;
    for (int sc : {1, 2, 4, 8, 16}) {
      if (sc > count && sc != 1) continue;
      if (c.shared > 1 && sc < 2 * c.shared) continue;  // a pipeline needs a stream besides its main one
      (void)msfv_batch_set_options(b, sc, c.graphs ? 1 : 0, c.shared);
      msfv_status st = batch_run(b, m, v, d_out, g_out);  // warm: captures graphs, builds shared launches
      if (st == MSFV_OK) st = msfv_batch_sync(b);
      if (st != MSFV_OK) return st;
      const auto t0 = std::chrono::steady_clock::now();
      st = batch_run(b, m, v, d_out, g_out);
      if (st == MSFV_OK) st = msfv_batch_sync(b);
      if (st != MSFV_OK) return st;
      const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      if (dt < best) {
        best = dt;
        best_s = sc;
        best_g = c.graphs;
        best_sh = c.shared;
      }
    }
  }
  msfv_status st = msfv_batch_set_options(b, best_s, best_g ? 1 : 0, best_sh);
  if (st != MSFV_OK) return st;
  if (streams_out) *streams_out = best_s;
  if (graphs_out) *graphs_out = best_g ? 1 : 0;
  if (shared_out) *shared_out = best_sh;
  return MSFV_OK;
}


// ---- serving ----------------------------------------------------------------

struct msfv_server {
  struct Req {
    int job = 0;
    Columns src;
    const double* m = nullptr;
    const double* v = nullptr;
    double* d = nullptr;
    double* g = nullptr;
    long long bytes = 0;                 // admission estimate of the request
    hipEvent_t ev_ready = nullptr;       // recorded on the caller's stream at submission
    hipEvent_t ev_start = nullptr, ev_end = nullptr;  // timing, on the job's stream
    std::chrono::steady_clock::time_point t_submit, t_done;
    double dev_start_ms = 0.0, dev_end_ms = 0.0;      // device times since the server's epoch
    int state = 0;  // 0 queued, 1 running, 2 done
    int waiters = 0;
    msfv_status st = MSFV_OK;
    std::string err;
  };
  struct Job {
    msfv_problem* p = nullptr;
    int max_sources = 0;
    long long resident = 0;  // device bytes the job's problem holds
    bool busy = false;
    long long pending = 0;   // request handed to the worker (0: none)
    std::condition_variable cv;
    std::thread th;
  };
  std::vector<std::unique_ptr<Job>> jobs;
  std::map<long long, Req> reqs;
  std::deque<long long> queue;
  std::vector<hipEvent_t> ev_sync, ev_timing;  // idle events
  std::mutex mu;
  std::condition_variable cv_done;
  bool stop = false;
  int max_inflight = 8;
  int running = 0;
  int device = 0;
  long long next_id = 1;
  long long budget = 0;        // bytes
  long long resident_total = 0;
  long long inflight_bytes = 0;
  long long peak_committed = 0;
  hipEvent_t epoch = nullptr;
  // statistics since the last reset
  std::vector<double> lat_ms;
  long long failed = 0, rejected = 0;
  bool have_first = false;
  std::chrono::steady_clock::time_point t_first, t_last;

  void worker(Job* j);
  void dispatch_locked();
  ~msfv_server() {
    {
      std::unique_lock<std::mutex> lk(mu);
      stop = true;
    }
    for (auto& j : jobs) j->cv.notify_all();
    for (auto& j : jobs)
      if (j->th.joinable()) j->th.join();
    for (auto e : ev_sync) (void)hipEventDestroy(e);
    for (auto e : ev_timing) (void)hipEventDestroy(e);
    if (epoch) (void)hipEventDestroy(epoch);
  }
};

namespace {

// Device bytes a problem holds (allocated capacity of every buffer).
long long problem_bytes(const msfv_problem* p) { return (long long)p->workspace_bytes(); }

// Bytes of a request beyond its job's resident state: the caller's buffers
// (m and g: N values each; v and D: Nr * Ns each).
long long request_bytes(const msfv_problem* p, int ns) {
  return 16LL * p->plan.ncell + 16LL * p->rec.count * ns;
}

// Allocate a job's source-count-dependent buffers for up to max_ns sources,
// so that requests never reallocate them (a hipFree would synchronise the
// device, stalling every other job).
msfv_status reserve_sources(msfv_problem* p, int max_ns) {
  const size_t ncs = size_t(p->plan.ncoarse) * max_ns;
  const size_t nd = size_t(std::max(1, p->rec.count)) * max_ns;
  HIP_OK(p->d_b.alloc(std::max(size_t(p->plan.ncoarse) * msfv::prolong_ldt(max_ns), 2 * ncs)));
  HIP_OK(p->d_t.alloc(2 * ncs));
  HIP_OK(p->d_D.alloc(nd));
  HIP_OK(p->d_v.alloc(nd));
  if (coarse_multi(p)) {
    HIP_OK(p->d_cg_ws.alloc(msfv::coarse_large_workspace(p->plan.ncv, 2 * max_ns) / sizeof(double) + 1));
    if (p->flags_cap < 2 * max_ns) {
      if (p->h_flags) HIP_OK(hipHostFree(p->h_flags));
      p->h_flags = nullptr;
      p->flags_cap = 0;
      HIP_OK(hipHostMalloc(reinterpret_cast<void**>(&p->h_flags), sizeof(int) * 6 * 2 * max_ns));
      p->flags_cap = 2 * max_ns;
    }
  }
  return MSFV_OK;
}

// Issue one request on its job's stream and wait for it (job worker thread,
// lock not held).
msfv_status serve_run(msfv_problem* p, msfv_server::Req& r, hipEvent_t epoch) {
  if (r.src.count != p->src.count || r.src.ptr != p->src.ptr || r.src.cell != p->src.cell ||
      r.src.val != p->src.val) {
    p->src = r.src;
    p->electrodes_ready = false;
    p->have_forward = false;
  }
  msfv_status st = ensure_ready(p);  // host tables of a new source set: this job's thread only
  if (st != MSFV_OK) return st;
  HIP_OK(hipStreamWaitEvent(p->stream, r.ev_ready, 0));  // inputs written on the caller's stream
  HIP_OK(hipEventRecord(r.ev_start, p->stream));
  st = forward_jtv_impl(p, r.m, r.v, r.d, r.g);
  if (st != MSFV_OK) return st;
  HIP_OK(hipEventRecord(r.ev_end, p->stream));
  HIP_OK(hipEventSynchronize(r.ev_end));
  float a = 0.f, b = 0.f;
  if (hipEventElapsedTime(&a, epoch, r.ev_start) == hipSuccess &&
      hipEventElapsedTime(&b, epoch, r.ev_end) == hipSuccess) {
    r.dev_start_ms = a;
    r.dev_end_ms = b;
  }
  return check_status(p);
}

}  // namespace

// Admit queued requests, first come first served: a request waits while its
// job is busy (a job's requests share its problem state and run in order),
// and no request is admitted past one that does not fit the memory budget,
// so a large request is not starved by smaller ones behind it.
void msfv_server::dispatch_locked() {
  for (auto it = queue.begin(); it != queue.end() && running < max_inflight;) {
    Req& r = reqs[*it];
    Job& j = *jobs[r.job];
    if (j.busy) {
      ++it;
      continue;
    }
    if (resident_total + inflight_bytes + r.bytes > budget) break;
    inflight_bytes += r.bytes;
    peak_committed = std::max(peak_committed, resident_total + inflight_bytes);
    ++running;
    j.busy = true;
    j.pending = *it;
    r.state = 1;
    it = queue.erase(it);
    j.cv.notify_one();
  }
}

void msfv_server::worker(Job* j) {
  (void)hipSetDevice(device);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    j->cv.wait(lk, [&] { return stop || j->pending != 0; });
    if (j->pending == 0) return;  // stopping, nothing handed over
    const long long id = j->pending;
    Req& r = reqs[id];  // map nodes stay put; a running request is never erased
    lk.unlock();
    msfv_status st = serve_run(j->p, r, epoch);
    std::string err = st == MSFV_OK ? std::string() : std::string(msfv_last_error());
    const auto t_done = std::chrono::steady_clock::now();
    lk.lock();
    r.st = st;
    r.err = std::move(err);
    r.t_done = t_done;
    r.state = 2;
    ev_sync.push_back(r.ev_ready);
    ev_timing.push_back(r.ev_start);
    ev_timing.push_back(r.ev_end);
    r.ev_ready = r.ev_start = r.ev_end = nullptr;
    lat_ms.push_back(std::chrono::duration<double, std::milli>(r.t_done - r.t_submit).count());
    if (st != MSFV_OK) ++failed;
    t_last = r.t_done;
    --running;
    inflight_bytes -= r.bytes;
    j->busy = false;
    j->pending = 0;
    dispatch_locked();
    cv_done.notify_all();
  }
}

msfv_status msfv_server_create(int max_inflight, double budget_bytes, msfv_server** out) {
  if (!out || max_inflight < 1 || max_inflight > 64) return fail(MSFV_EINVAL, "max_inflight outside [1, 64]");
  *out = nullptr;
  std::unique_ptr<msfv_server> s(new msfv_server());
  s->max_inflight = max_inflight;
  HIP_OK(hipGetDevice(&s->device));
  if (budget_bytes > 0) {
    s->budget = (long long)budget_bytes;
  } else {
    size_t free_b = 0, total_b = 0;
    HIP_OK(hipMemGetInfo(&free_b, &total_b));
    s->budget = (long long)total_b;
  }
  HIP_OK(hipEventCreate(&s->epoch));
  HIP_OK(hipEventRecord(s->epoch, nullptr));
  HIP_OK(hipEventSynchronize(s->epoch));
  *out = s.release();
  return MSFV_OK;
}

void msfv_server_destroy(msfv_server* s) {
  if (!s) return;
  (void)msfv_server_drain(s);
  delete s;
}

msfv_status msfv_server_add_job(msfv_server* s, msfv_problem* p, int max_sources, int* job) {
  if (!s || !p || !job) return fail(MSFV_EINVAL, "null argument");
  if (max_sources < 1) return fail(MSFV_EINVAL, "max_sources must be at least 1");
  {
    std::unique_lock<std::mutex> lk(s->mu);
    for (auto& j : s->jobs)
      if (j->p == p) return fail(MSFV_EINVAL, "problem already registered");
  }
  if (p->rec.count <= 0) return fail(MSFV_ESTATE, "job problem has no receivers");
  HIP_OK(hipStreamSynchronize(p->stream));
  {
    // estimate before reserving: the coarse vectors (3 Nc) and data buffers
    // (2 Nr) of max_sources sources on top of what the problem holds now
    const long long est = problem_bytes(p) + 8LL * (3LL * p->plan.ncoarse + 2LL * p->rec.count) * max_sources;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->resident_total + est > s->budget)
      return fail(MSFV_ENOMEM, "the job's resident state exceeds the server's memory budget");
  }
  msfv_status st = reserve_sources(p, max_sources);
  if (st != MSFV_OK) return st;
  std::unique_ptr<msfv_server::Job> j(new msfv_server::Job());
  j->p = p;
  j->max_sources = max_sources;
  j->resident = problem_bytes(p);
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->resident_total + j->resident > s->budget)
    return fail(MSFV_ENOMEM, "the job's resident state exceeds the server's memory budget");
  s->resident_total += j->resident;
  msfv_server::Job* raw = j.get();
  s->jobs.push_back(std::move(j));
  raw->th = std::thread([s, raw] { s->worker(raw); });
  *job = int(s->jobs.size()) - 1;
  return MSFV_OK;
}

msfv_status msfv_server_request_bytes(msfv_server* s, int job, int ns, long long* resident,
                                      long long* request) {
  if (!s) return fail(MSFV_EINVAL, "null server");
  std::unique_lock<std::mutex> lk(s->mu);
  if (job < 0 || job >= int(s->jobs.size())) return fail(MSFV_EINVAL, "unknown job");
  const msfv_server::Job& j = *s->jobs[job];
  if (resident) *resident = j.resident;
  if (request) *request = request_bytes(j.p, ns);
  return MSFV_OK;
}

msfv_status msfv_server_submit(msfv_server* s, int job, int ns, const int* ptr, const int* cell,
                               const double* val, const double* m, const double* v, double* d_out,
                               double* g_out, void* caller_stream, long long* req) {
  if (!s || !m || !v || !d_out || !g_out || !req) return fail(MSFV_EINVAL, "null argument");
  msfv_problem* p = nullptr;
  int max_sources = 0;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    if (job < 0 || job >= int(s->jobs.size())) return fail(MSFV_EINVAL, "unknown job");
    p = s->jobs[job]->p;
    max_sources = s->jobs[job]->max_sources;
  }
  if (ns < 1 || ns > max_sources)
    return fail(MSFV_EINVAL, "request source count outside [1, the job's max_sources]");
  msfv_server::Req r;
  msfv_status st = check_columns(p, ns, ptr, cell, val, &r.src);
  if (st != MSFV_OK) return st;
  r.job = job;
  r.m = m;
  r.v = v;
  r.d = d_out;
  r.g = g_out;
  r.bytes = request_bytes(p, ns);
  {
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->resident_total + r.bytes > s->budget) {
      ++s->rejected;
      return fail(MSFV_ENOMEM, "the request does not fit the server's memory budget even alone");
    }
    if (!s->ev_sync.empty()) {
      r.ev_ready = s->ev_sync.back();
      s->ev_sync.pop_back();
    }
    for (hipEvent_t* e : {&r.ev_start, &r.ev_end})
      if (!s->ev_timing.empty()) {
        *e = s->ev_timing.back();
        s->ev_timing.pop_back();
      }
  }
  auto give_back = [&]() {
    std::unique_lock<std::mutex> lk(s->mu);
    if (r.ev_ready) s->ev_sync.push_back(r.ev_ready);
    if (r.ev_start) s->ev_timing.push_back(r.ev_start);
    if (r.ev_end) s->ev_timing.push_back(r.ev_end);
  };
  hipError_t e = hipSuccess;
  if (!r.ev_ready) e = hipEventCreateWithFlags(&r.ev_ready, hipEventDisableTiming);
  if (e == hipSuccess && !r.ev_start) e = hipEventCreate(&r.ev_start);
  if (e == hipSuccess && !r.ev_end) e = hipEventCreate(&r.ev_end);
  // the request's inputs are ordered after the caller's work on its stream
  if (e == hipSuccess) e = hipEventRecord(r.ev_ready, static_cast<hipStream_t>(caller_stream));
  if (e != hipSuccess) {
    give_back();
    return fail(MSFV_EDEVICE, std::string("msfv_server_submit: ") + hipGetErrorString(e));
  }
  r.t_submit = std::chrono::steady_clock::now();
  {
    std::unique_lock<std::mutex> lk(s->mu);
    const long long id = s->next_id++;
    if (!s->have_first) {
      s->have_first = true;
      s->t_first = r.t_submit;
    }
    s->reqs.emplace(id, std::move(r));
    s->queue.push_back(id);
    *req = id;
    s->dispatch_locked();
  }
  return MSFV_OK;
}

msfv_status msfv_server_wait(msfv_server* s, long long req, double* latency_ms, double* dev_start_ms,
                             double* dev_end_ms) {
  if (!s) return fail(MSFV_EINVAL, "null server");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(req);
  if (it == s->reqs.end()) return fail(MSFV_EINVAL, "unknown request");
  ++it->second.waiters;  // keeps the entry until this waiter has read it
  s->cv_done.wait(lk, [&] { return s->reqs.find(req)->second.state == 2; });
  it = s->reqs.find(req);
  msfv_server::Req& r = it->second;
  const msfv_status st = r.st;
  const std::string err = r.err;
  if (latency_ms) *latency_ms = std::chrono::duration<double, std::milli>(r.t_done - r.t_submit).count();
  if (dev_start_ms) *dev_start_ms = r.dev_start_ms;
  if (dev_end_ms) *dev_end_ms = r.dev_end_ms;
  if (--r.waiters == 0) s->reqs.erase(it);
  lk.unlock();
  if (st != MSFV_OK) return fail(st, err);
  return MSFV_OK;
}

msfv_status msfv_server_drain(msfv_server* s) {
  if (!s) return fail(MSFV_EINVAL, "null server");
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] { return s->queue.empty() && s->running == 0; });
  // forget completed requests nobody waits for
  for (auto it = s->reqs.begin(); it != s->reqs.end();)
    it = (it->second.state == 2 && it->second.waiters == 0) ? s->reqs.erase(it) : std::next(it);
  return MSFV_OK;
}

msfv_status msfv_server_stats(msfv_server* s, msfv_serve_stats* out, int reset) {
  if (!s || !out) return fail(MSFV_EINVAL, "null argument");
  std::unique_lock<std::mutex> lk(s->mu);
  std::memset(out, 0, sizeof *out);
  std::vector<double> v = s->lat_ms;
  std::sort(v.begin(), v.end());
  out->completed = (long long)v.size();
  out->failed = s->failed;
  auto pct = [&](double q) {
    if (v.empty()) return 0.0;
    const double pos = q * double(v.size() - 1);
    const size_t i = size_t(pos);
    const double f = pos - double(i);
    return i + 1 < v.size() ? v[i] * (1.0 - f) + v[i + 1] * f : v[i];
  };
  out->p50_ms = pct(0.50);
  out->p90_ms = pct(0.90);
  out->p99_ms = pct(0.99);
  double sum = 0.0;
  for (double x : v) sum += x;
  out->mean_ms = v.empty() ? 0.0 : sum / double(v.size());
  out->max_ms = v.empty() ? 0.0 : v.back();
  if (s->have_first && !v.empty()) {
    out->span_s = std::chrono::duration<double>(s->t_last - s->t_first).count();
    out->throughput = out->span_s > 0 ? double(v.size()) / out->span_s : 0.0;
  }
  out->rejected = s->rejected;
  out->budget_bytes = double(s->budget);
  out->resident_bytes = double(s->resident_total);
  out->peak_committed_bytes = double(s->peak_committed);
  if (reset) {
    s->lat_ms.clear();
    s->failed = 0;
    s->rejected = 0;
    s->have_first = false;
    s->peak_committed = s->resident_total + s->inflight_bytes;
  }
  return MSFV_OK;
}

}  // extern "C"
