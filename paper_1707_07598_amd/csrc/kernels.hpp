// Launchers of the gfx950 kernels of the MSFV path (implemented in
// kernels.hip, wave_kernels.hip and coarse_kernels.hip).  All pointers are device pointers; every launcher enqueues
// on ``stream`` and returns the hipError_t of the launch.
#pragma once
#include <vector>

#include <hip/hip_runtime.h>

#include <algorithm>

#include "plan.hpp"

namespace msfv {

struct GridInfo {
  int n[3];
  int s1, s2;  // cell strides of axes 1 and 2
};

// status words written by the kernels
enum StatusSlot {
  kStNonfinite = 0,
  kStLocalNoconv = 1,
  kStReserved = 2,  // local CG iteration counts are kept per entity
  kStCoarseNoconv = 3,
  kStCoarseMaxIt = 4,
  kStCoarseRes = 6,  // two words: largest (||r|| / ||b||)^2 of a coarse solve, as double bits
  kStCount = 8
};

// Raise the residual maximum in status[slot] to rel2 = (||r|| / ||b||)^2 of
// a finished solve.  The bit patterns of non-negative doubles order like
// their values, so an unsigned 64-bit maximum keeps the largest; a NaN
// counts as +inf.
__device__ __forceinline__ void note_residual(int* status, int slot, double rel2) {
  if (!(rel2 >= 0.0)) rel2 = __builtin_huge_val();
  atomicMax(reinterpret_cast<unsigned long long*>(status + slot),
            static_cast<unsigned long long>(__double_as_longlong(rel2)));
}

struct LocalParams {
  const EntDesc* ents = nullptr;  // entities solved by this launch
  int nent = 0;
  const EntDesc* recv = nullptr;  // entities receiving adjoint loads (next lower kind)
  GridInfo g{};
  const double* m = nullptr;
  const double* sig = nullptr;  // exp(m), where a kernel reads it instead of forming it
  const int* prow = nullptr;
  const int* pcol = nullptr;
  double* pval = nullptr;
  double* kent = nullptr;
  double rtol = 1e-13;
  int maxit = 1000;
  int prescribe = 0;   // forward: Lagrange values instead of a solve
  int* status = nullptr;
  int sig_cap = 0;     // LDS doubles reserved for the closure conductivities
  int nu_cap = 0;      // largest own-cell count in this launch
  int lane_cap = 0;    // largest own-cell plane over the two lane axes
  int col_cap = 0;     // largest own-cell column along the third axis
  int nc_cap = 0;      // largest corner count
  int plane_cap = 0;   // largest zero-padded plane buffer (doubles per wave)
  int line_cap = 0;    // edges: longest closure line (cells) of the launch
  // adjoint
  const double* t = nullptr;
  const double* lam = nullptr;
  int ncoarse = 0;
  int ns = 0;
  const double* inbuf = nullptr;   // loads received by these entities
  double* outbuf = nullptr;        // loads pushed to the receivers
  const int* eidx = nullptr;       // electrode index per entity electrode slot
  const int* eloc = nullptr;       // own-cell index of that electrode
  const double* sload = nullptr;   // direct loads per electrode and corner (8 each)
  double* W = nullptr;             // 3*N flux weights
  int solve_adj = 1;               // 0: flux-derivative (G) term only
  int push = 1;                    // 1: push loads to lower entities
  int* ent_it = nullptr;                  // per entity: largest CG iteration count of its corners
  double* ent_res = nullptr;              // per entity, 8 slots (corners or passes): final (||r|| / ||b||)^2
  unsigned long long* ent_work = nullptr; // per entity, if set: += CG cell-iterations (iterations x own cells)
  double* mu_scratch = nullptr;           // adjoint: per entity 8 * nu_cap doubles (local adjoint solutions)
  int uni_cap = 0;                        // wave kernels: doubles of the shared plane-buffer region
  const double* dm = nullptr;             // tangent passes: direction of the model perturbation
  double* dpval = nullptr;                // tangent passes: dS_k values (CSR of S_k)
  const int* ent_list = nullptr;          // if set: workgroup b solves entity ent_list[b] of ents
  int lagrange = 0;                       // edges of multi-instance launches: Lagrange boundary values
  // Multi-instance launches (many problems, one launch): item i of the nent
  // items is entity items[i].y of the problem whose parameters are
  // multi[items[i].x]; a fixed grid of workgroups strides over the items.
  const LocalParams* multi = nullptr;
  const int2* items = nullptr;
};

// The entity of this workgroup (per-entity outputs are indexed by it).
__device__ __forceinline__ int ent_index(const LocalParams& a) {
  return a.ent_list ? a.ent_list[blockIdx.x] : int(blockIdx.x);
}

hipError_t launch_check_finite(const double* m, long long n, int* status, hipStream_t s);
hipError_t launch_edge_fwd(const LocalParams& p, int lagrange, hipStream_t s);
hipError_t launch_local_fwd(const LocalParams& p, int kind_rmax, hipStream_t s);
hipError_t launch_edge_adj(const LocalParams& p, int lagrange, hipStream_t s);
hipError_t launch_local_adj(const LocalParams& p, int kind_rmax, hipStream_t s);
// Zero `bytes` (a multiple of 4) / copy n doubles with plain kernels, so that
// the per-call sequence holds only kernel launches (safe to capture in a graph).
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);
hipError_t launch_copy(double* dst, const double* src, long long n, hipStream_t s);
hipError_t launch_set_ones(const int* idx, int n, double* out, hipStream_t s);
// A_k as CSR (kval) and as 27 diagonals of the coarse grid (kdia[o*ldk + row],
// o = (dx+1) + 3(dy+1) + 9(dz+1), ldk = coarse_ldk(nc)); dslot maps each CSR
// nonzero to its slot.
hipError_t launch_kassemble(const int* kcptr, const int* kcidx, const int* dslot, const double* kent,
                            double* kval, double* kdia, int nnz, hipStream_t s);
// Row stride of the diagonal storage used by the coarse solver (rows padded
// with zeros to a multiple of its workgroup size).
int coarse_ldk(int nc);
// Aggregates of the two-level coarse preconditioner: boxes of b[0] x b[1] x
// b[2] coarse vertices, na3[k] boxes per axis, na <= 64 in all.
struct CoarseDefl {
  int b[3] = {1, 1, 1};
  int na3[3] = {1, 1, 1};
  int na = 0;
  bool ok = false;              // fits the kernels' LDS budgets
  const double* einv = nullptr; // device, na x na: (Z^T A_k Z)^-1 over the free vertices
  const int* arows = nullptr;   // device: aggregate offsets (na + 1), then the vertices by aggregate
};
CoarseDefl coarse_defl_plan(const int ncv[3]);
// the same boxes for the multi-launch solver (E^-1 in LDS only for the setup)
CoarseDefl coarse_defl_plan_large(const int ncv[3]);
// Host table for CoarseDefl::arows: offsets of each aggregate's vertices
// (na + 1 entries), then the vertex ids aggregate by aggregate, x fastest
// within a box.
std::vector<int> coarse_defl_rows(const CoarseDefl& d, const int ncv[3]);
// einv = (Z^T A_k Z)^-1 (one workgroup); a non-positive pivot counts as a
// non-converged coarse solve in status.
hipError_t launch_coarse_defl_setup(const double* kdia, const int ncv[3], const CoarseDefl& d,
                                    double* einv, int* status, hipStream_t s);
// Coarse systems too large for one workgroup take the multi-launch solver:
// PCG over all columns, three launches per iteration (five with the
// two-level correction, when defl is given), and the host polls the stop
// flags every few iterations (so the call blocks until the solve ends).
// workspace: coarse_large_workspace bytes of device memory; host_flags: 6*ns
// ints of pinned host memory.
bool coarse_is_large(const int ncv[3]);
size_t coarse_large_workspace(const int ncv[3], int ns);
hipError_t launch_coarse_pcg_large(const double* kdia, const int ncv[3], const double* rhs, double* x,
                                   int ns, double rtol, int maxit, const CoarseDefl* defl, void* workspace,
                                   int* host_flags, int* status, unsigned long long* work, hipStream_t s);
// PCG on A_k with vertex 0 fixed, one workgroup per column of rhs; Jacobi
// preconditioned, plus the aggregate correction when defl is given.
hipError_t launch_coarse_pcg(const double* kdia, const int ncv[3], const double* rhs, double* x,
                             int ncol, double rtol, int maxit, const CoarseDefl* defl, int* status,
                             unsigned long long* work, hipStream_t s);
// energy blocks of the entities of p.ents (corner count <= p.nc_cap <= 8)
// from the S_k values in p.pval and p.sig = exp(m), into p.kent: A_k of a
// frozen basis (wave_kernels.hip)
hipError_t launch_energy_frozen(const LocalParams& p, hipStream_t s);
// Multi-instance local solves.  A class is the kernel variant that
// launch_local_* (or launch_wave_full / launch_wave_faces, for the full
// blocks and faces) would pick for a problem's entity list; items of one
// class from many problems run in one launch of a fixed grid.  p carries multi, items, nent and the largest caps
// over the problems of the class (for the LDS size).
enum LocalClass {
  kClassNone = 0,
  kClassWave441 = 1, kClassWave443, kClassWave447, kClassWave481, kClassWave483, kClassWave487,
  kClassFull3, kClassFull7,
  kClassFaces3, kClassFaces7,  // faces, the full 3 x 3 (7 x 7) ones with their shape fixed
  kClassLocalFirst = 16  // + index of the generic variant
};
int local_class(const LocalParams& p);      // class of a problem's launch (caps of p)
int full_class(int u);                      // class of full u^3 blocks
int faces_class(int u);                     // class of faces whose full ones have u x u own cells
// uni_cap a problem's parameters must carry in a launch of class klass
int local_class_uni_cap(const LocalParams& p, int klass);
hipError_t launch_local_multi(const LocalParams& p, int klass, bool adj, hipStream_t s);
hipError_t launch_edge_multi(const LocalParams& p, bool adj, hipStream_t s);
// wave-kernel classes (wave_kernels.hip)
int wave_class(const LocalParams& p);
int wave_class_uni_cap(const LocalParams& p, int klass);
hipError_t launch_wave_multi(const LocalParams& p, int klass, bool adj, hipStream_t s);
// wave-per-corner local solves (wave_kernels.hip)
bool wave_path_fits(const LocalParams& p);
hipError_t launch_wave_local(const LocalParams& p, bool adj, hipStream_t s);
// the same for full dual blocks of u^3 own cells (u = 3 or 7) listed in
// p.ent_list, with their geometry fixed at compile time
hipError_t launch_wave_full(const LocalParams& p, int u, bool adj, hipStream_t s);
// forward local solves of all dual blocks of p.ent_list in one launch (caps
// within the wave path): the full u^3 ones (u = 7, or u = 3 when no column
// exceeds 3 cells) through the body with their geometry fixed, the others
// through the general body
hipError_t launch_wave_blocks(const LocalParams& p, int u, hipStream_t s);
// and for faces (one cell a lane, caps within one wavefront): the full faces
// of u x u own cells (u = 3 or 7, bounded by vertex planes on both open
// axes) through bodies with their geometry fixed, one for each plane axis,
// the others through the general body, all in one launch
hipError_t launch_wave_faces(const LocalParams& p, int u, bool adj, hipStream_t s);
// out[slot_dst[s] + j*nc] = sum_e w[e] * pval[pidx[e]] * (colw ? colw[j*colw_ld + col[e]] : 1)
// for slot s and column j < ncol (one thread each).
hipError_t launch_gather_slots(const int* slot_dst, const int* slot_ptr, const int* ent_pidx,
                               const double* ent_w, const int* ent_col, const double* colw,
                               int colw_ld, const double* pval, double* out, int nslot,
                               int ncol, int nc, hipStream_t s);
hipError_t launch_data(const int* rptr, const int* rcell, const double* rval, int nr, int ns,
                       const int* prow, const int* pcol, const double* pval, const double* t,
                       int nc, double* D, hipStream_t s, int accumulate = 0);
// u_j = S_k t_j (N values per source, column j contiguous) on the vertex
// grid ncv; scratch holds nc * prolong_ldt(ns) doubles (the coefficients
// vertex by vertex)
int prolong_ldt(int ns);
hipError_t launch_prolong(const int* prow, const int* pcol, const double* pval, const double* t,
                          const int ncv[3], int ns, long long ncell, double* u, double* scratch, hipStream_t s);
hipError_t launch_sload(int nelec, const int* ecell, const int* rptr, const int* ridx,
                        const double* rw, const int* sptr, const int* sidx, const double* sw,
                        const int* prow, const int* pcol, const double* t, const double* lam,
                        const double* v, int nc, int ns, int nr, double* sload, hipStream_t s);
// grad from the per-flux weights W (3N) with sig = exp(m)
hipError_t launch_gfinal(const double* sig, const double* W, GridInfo g, long long ncell, double* grad,
                         hipStream_t s);
// dst = m, sig = exp(m), status flag for non-finite entries
hipError_t launch_prep_model(double* dst, double* sig, const double* src, long long n, int* status,
                             hipStream_t s);
// Sensitivity passes (forward-mode J and the fixed-basis variants):
// tangent edge basis and energy blocks (kent <- dK_E, dpval <- dS on own cells)
hipError_t launch_edge_tan(const LocalParams& p, int lagrange, hipStream_t s);
// tangent face / dual-block basis and energy blocks (wave_kernels.hip)
hipError_t launch_wave_tan(const LocalParams& p, hipStream_t s);
// the same for any entity size: the wave kernels where they fit, else the
// workgroup-per-entity kernels (kernels.hip)
hipError_t launch_local_tan(const LocalParams& p, hipStream_t s);
// y_j = (dA/dm . dm) u_j for all ns columns of u (N each)
hipError_t launch_dAu(const double* m, const double* dm, GridInfo g, long long ncell, int ns,
                      const double* u, double* y, hipStream_t s);
// W_k(i) = -sum_j (u_j(i) - u_j(i+e_k)) (z_j(i) - z_j(i+e_k))
hipError_t launch_wfixed(GridInfo g, long long ncell, int ns, const double* u, const double* z, double* W,
                         hipStream_t s);
// b_j = scale * S_k^T y_j through the column lists of S_k
hipError_t launch_restrict(const int* cptr, const int* cidx, const int* ccell, const double* pval,
                           const double* y, int nc, int ns, long long ncell, double scale, double* b,
                           hipStream_t s);
// rhs_j -= dK t_j with dK in 27-diagonal storage
hipError_t launch_coarse_dk_sub(const double* kd, int ldk, const int ncv[3], int ns, const double* t,
                                double* rhs, hipStream_t s);
hipError_t launch_residual(const double* D, const double* dobs, double* v, long long n,
                           double* phi, hipStream_t s);

}  // namespace msfv
