// Internal declarations of the stfdfd library (host plans, device layouts, launchers).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <complex>
#include <cstdint>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/stfdfd.h"

namespace stf {

using cd = std::complex<double>;

struct Error : std::runtime_error {
  stf_status code;
  Error(stf_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define STF_REQUIRE(cond, msg)                                        \
  do {                                                                \
    if (!(cond)) throw ::stf::Error(STF_EINVAL, std::string(msg));    \
  } while (0)

#define HIP_CHECK(expr)                                                                    \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      throw ::stf::Error(e_ == hipErrorOutOfMemory ? STF_ENOMEM : STF_EDEVICE,             \
                         std::string(#expr) + ": " + hipGetErrorString(e_));               \
  } while (0)

// Per-kernel timing.  While a timer is installed on the calling thread, every
// launch through STF_LAUNCH asks it for a start and a stop event, which the
// runtime records as part of that kernel's own dispatch (hipExtLaunchKernelGGL),
// so that their interval is the kernel's execution alone, as in a kernel trace;
// without a timer (or when the timer declines, e.g. during graph capture) the
// launch is a plain one.
struct KernelTimer {
  virtual bool events(hipStream_t st, hipEvent_t* start, hipEvent_t* stop) = 0;

 protected:
  ~KernelTimer() = default;
};
extern thread_local KernelTimer* t_kernel_timer;

#define STF_LAUNCH(K, GRID, BLOCK, SHMEM, STREAM, ...)                                       \
  do {                                                                                     \
    hipEvent_t stf_t0_ = nullptr, stf_t1_ = nullptr;                                       \
    if (::stf::t_kernel_timer && ::stf::t_kernel_timer->events((STREAM), &stf_t0_, &stf_t1_)) \
      hipExtLaunchKernelGGL(K, GRID, BLOCK, SHMEM, STREAM, stf_t0_, stf_t1_, 0u, __VA_ARGS__); \
    else                                                                                   \
      hipLaunchKernelGGL(K, GRID, BLOCK, SHMEM, STREAM, __VA_ARGS__);                      \
  } while (0)

// ---------------------------------------------------------------------------
// Host plan: stretch arrays, partition, nested dissection (host_plan.cpp)
// ---------------------------------------------------------------------------

// 1D coupling coefficients of one axis of a domain: w[t] couples node t to t-1,
// e[t] couples t to t+1 (Eq. (9) discretised: 1/(d^2 s[t] s[t -/+ 1/2])).
struct AxisCoef {
  std::vector<cd> w, e;
};

struct SubDesc {
  int kx, ky;
  int ox0, oy0, nxl, nyl;   // Omega_k: global node box [ox0, ox0+nxl) x [oy0, oy0+nyl)
  int ix0, ix1, iy0, iy1;   // I_k (global node ranges, half-open)
  AxisCoef cx, cy;          // local coupling coefficients
  int shape;                // index of the symbolic plan
};

// One front of the nested-dissection elimination tree of a local grid.
struct SymFront {
  int p = 0, q = 0;         // separator (fully summed) size, update-set size
  int parent = -1;          // index in the shape's front list
  int depth = 0;            // root = 0
  int var_off = 0;          // vars[var_off .. var_off+p+q): local node ids, separator first
  int cmap_off = 0;         // cmap[cmap_off .. +q): position of each update var in the parent front
  int ent_off = 0, ent_cnt = 0;   // original matrix entries assembled into this front
  int child_off = 0, nchild = 0;  // children[child_off ..)
  int sx0 = 0, sy0 = 0, sw = 1;   // the separator is the local box at (sx0, sy0) of width
                                  // sw, its nodes listed row by row (vars[var_off + i] =
                                  // sx0 + i % sw + (sy0 + i / sw) * nxl)
};

// Packed original entry: front row, front column, local node, stencil direction.
// dir: 0 centre, 1 west (t-1), 2 east (t+1), 3 south (u-1), 4 north (u+1); the value
// is row `node`'s coefficient towards its neighbour in that direction.
struct SymEntry {
  int32_t rc;      // row | (col << 16)
  int32_t nd;      // node * 8 + dir
};

struct SymShape {
  int nxl = 0, nyl = 0, leaf = 0;
  std::vector<SymFront> fronts;    // preorder (parents before children)
  std::vector<int> vars, cmap, children;
  std::vector<SymEntry> ents;
  int max_depth = 0, max_front = 0;
  int64_t factor_entries = 0, front_entries = 0, vec_entries = 0;
  double lu_flops = 0.0;
};

struct GlobalAxes {
  std::vector<cd> sx, sxh, sy, syh;   // s at nodes, s at half points i-1/2 (n+1 entries)
  AxisCoef cx, cy;
};

struct Plan {
  stf_params prm;
  GlobalAxes g;
  std::vector<SubDesc> subs;
  std::vector<std::shared_ptr<const SymShape>> shapes;
  // Per-axis cover tables for the sum of local fields: for global index g, up to two
  // (block, local coordinate) pairs; block -1 = none.
  std::vector<int4> cover_x, cover_y;
};

void validate_params(const stf_params& p);
stf_params normalized(const stf_params& p);
GlobalAxes build_global_axes(const stf_params& p);
std::vector<SubDesc> build_partition(const stf_params& p, const GlobalAxes& g);
std::shared_ptr<SymShape> build_symbolic(int nxl, int nyl, int leaf);
void build_cover(const stf_params& p, const std::vector<SubDesc>& subs, std::vector<int4>& cx,
                 std::vector<int4>& cy);
// Builds the whole host plan; shape_cache (may be null) memoises symbolic plans.
Plan build_plan(const stf_params& p,
                std::map<std::tuple<int, int, int>, std::shared_ptr<const SymShape>>* shape_cache);
stf_plan_info plan_info(const Plan& pl);

// ---------------------------------------------------------------------------
// Device layouts (shared by host launch code and kernels)
// ---------------------------------------------------------------------------

// Several problems can share one set of device arrays (a batch): problem p's
// nodes are then the segment [gbase, gbase + nx*ny) of concatenated global
// vectors, so every node array is indexed gbase + y*gnx + x.
struct SubDev {
  int ox0, oy0, nxl, nyl;
  int ix0, ix1, iy0, iy1;
  int cx_off, cy_off;       // offsets of (w, e) pairs in the local coefficient arrays
  long long u_off;          // offset of the local field (nxl*nyl elements)
  long long gbase;          // first node of the subdomain's problem in global vectors
  int gnx;                  // that problem's nx
  int prob;                 // that problem's index in the set
};

// Front instances are stored in tree-level order (deepest level last within
// the array's level ranges, largest fronts first within a level), so a level
// is the contiguous range [first, first + n).  The children's vector offsets
// and maps are embedded so that the sweeps read one descriptor per front.
struct FrontDev {
  long long fac_off;        // element offset of the m x m front (column-major)
  long long lpk_off;        // element offset of the packed forward operator
  long long upk_off;        // element offset of the packed backward operator
  int vec_off;              // element offset of the front vector (m elements)
  int piv_off;              // offset of the p pivot entries
  int p, q;
  int sub;                  // subdomain
  int var_off, cmap_off;    // into the concatenated vars / cmap arrays
  int ent_off, ent_cnt;     // into the concatenated entries
  int parent;               // instance index or -1
  int child_off, nchild;    // into the instance children array (nchild <= 2)
  int cvec[2];              // children: vec_off + p (start of their update parts)
  int ccmap[2];             // children: cmap_off
  int cq[2];                // children: q
  // The separator's global node box (origin gx0, gy0; width sw; row by row) and
  // the subdomain's I_k: row i < p of the front is global node
  // (gx0 + i % sw, gy0 + i / sw), restricted to I_k by the forward sweep
  // without a load of its local index.
  int gx0, gy0, sw;
  int ix0, ix1, iy0, iy1;
  long long gbase;          // the problem's first node in global vectors
  int gnx;                  // the problem's nx
  int prob;                 // the problem's index in the set
};

// Per problem of a set, for the sum of local fields into global vectors.
struct ScatDev {
  int sub0, px, nx, ny;     // first subdomain, subdomain columns, grid
  int cx_off, cy_off;       // offsets into the concatenated cover tables
  long long gbase;          // first node in global vectors
  int gc_off;               // offset of the problem's global coupling arrays (cxw|cxe|cyw|cye)
  int pad;
};

// Right-hand sides swept together (1..MAX_RHS): each has its own global input
// and output vector and its own copy of the front-vector and local-field
// workspaces, at fixed strides; the factors are read once for all of them.
constexpr int MAX_RHS = 4;
struct RhsSet {
  int nr = 1;
  long long vec_stride = 0;            // elements between RHS copies of the front vectors
  long long u_stride = 0;              // elements between RHS copies of the local fields
  const double2* v[MAX_RHS] = {};      // restricted sources (global, FP64)
  double2* z[MAX_RHS] = {};            // round outputs (global, FP64)
};

// One system of a batched solve (a problem and one of its right-hand sides):
// the segment [off, off + n) of every batch vector, systems slot-major
// (s = slot * nprob + problem).
struct SysDev {
  long long off;            // first entry in the batch vectors
  long long koff;           // first node of its problem in the concatenated node arrays
  int n, nx, ny;            // entries (nx * ny) and grid
  int gc;                   // offset of its problem's coupling arrays (cxw | cxe | cyw | cye)
  int present;              // 0: a slot beyond its problem's right-hand sides
  int tile0;                // first 64 x 4 stencil tile
  int blk0[4], nblk[4];     // first block and block count for chunks of 256 << c entries
};

// Kernel classes for timing (match STF_K_* in stfdfd.h).
enum KClass {
  K_ASSEMBLE = STF_K_ASSEMBLE, K_STENCIL = STF_K_STENCIL, K_FRONT_ASM = STF_K_FRONT_ASM,
  K_FRONT_LU = STF_K_FRONT_LU, K_SWEEP_FWD = STF_K_SWEEP_FWD, K_SWEEP_BWD = STF_K_SWEEP_BWD,
  K_SCATTER = STF_K_SCATTER, K_ARNOLDI = STF_K_ARNOLDI, K_UPDATE = STF_K_UPDATE,
  K_NN = STF_K_NN
};

// ---------------------------------------------------------------------------
// Launchers (kernels_*.hip).  All are asynchronous on `st`.
// ---------------------------------------------------------------------------

// node k0^2 * eps_bar from the cell map (Eq. (3)).
void launch_node_keps(hipStream_t st, const double2* cells, double2* keps, int nx, int ny,
                      double k0sq);
// y_s = A x_s for nr (<= MAX_RHS) vectors in one launch (the coefficients
// read once per node for all of them).
struct StencilSet {
  const double2* x[MAX_RHS] = {};
  double2* y[MAX_RHS] = {};
};
void launch_stencil_set(hipStream_t st, int nr, const StencilSet& S, const double2* keps,
                        const double2* cxw, const double2* cxe, const double2* cyw,
                        const double2* cye, int nx, int ny);
// r_s = b_s - A x_s for nr (<= MAX_RHS) vectors, then out_s[0] = |r_s|^2 (and
// host_out_s[0] when given: device-visible host memory) from per-block
// partials (partial_s: one double per 256-node block); two launches in all.
struct ResidualSet {
  const double2* x[MAX_RHS] = {};
  const double2* b[MAX_RHS] = {};
  double2* r[MAX_RHS] = {};
  double* partial[MAX_RHS] = {};
  double* out[MAX_RHS] = {};
  double* host_out[MAX_RHS] = {};
};
void launch_residual_set(hipStream_t st, int nr, const ResidualSet& S, const double2* keps,
                         const double2* cxw, const double2* cxe, const double2* cyw,
                         const double2* cye, int nx, int ny);
// y = A x  (mode 0) or r = b - A x with per-block partial |r|^2 (mode 1).
void launch_stencil(hipStream_t st, int mode, const double2* x, const double2* b, double2* y,
                    const double2* keps, const double2* cxw, const double2* cxe,
                    const double2* cyw, const double2* cye, int nx, int ny, double* partial,
                    int* nblocks_out);
int stencil_partial_blocks(int nx, int ny);
// out[0] = sum partial[0..n)  (single block, fixed order).
void launch_reduce_sum(hipStream_t st, const double* partial, int n, double* out);
// Power through the grid line between node rows (axis 1) or columns (axis 0)
// index and index + 1, nodes [lo, hi) along it; out: one device double.  The
// caller checks 0 <= index, index + 1 < ny (nx), 0 <= lo <= hi <= nx (ny).
void launch_line_flux(hipStream_t st, const double2* e, int nx, int axis, int index, int lo, int hi,
                      double k0, double dx, double dy, double* out);
// F[a] of the near-to-far-field transform at angle phis[a] (device) over the
// rectangle through the half-node lines around node box [i0, i1] x [j0, j1]
// (the caller checks 0 <= i0 < i1, i1 + 1 < nx, likewise j).
void launch_far_field(hipStream_t st, const double2* e, int nx, int i0, int i1, int j0, int j1,
                      double dx, double dy, double k0, const double* phis, int nang, double2* F);
// nonzero flag if any of n doubles is not finite (flag must be zeroed first).
void launch_check_finite(hipStream_t st, const double* a, long long n, int* flag);

// Multifrontal, per tree level; T = double2 (c128) or float2 (c64).
struct LevelArgs {
  const FrontDev* fronts;       // instance descriptors (level order)
  int first;                    // first front of this level
  int nlevel;                   // number of fronts in the level
  const SubDev* subs;
  const int* vars;
  const int* cmap;
  const SymEntry* ents;
  const int* children;
  const double2* keps;          // global k0^2 eps_bar (concatenated over the set's problems)
  const double2* lcoef;         // local coupling coefficients
  const int* pact;              // sweeps: per problem, nonzero while one of its right-hand
                                // sides is active (null = all); fronts of others are skipped
  const int* flist;             // sweeps: front instances [first, first + nlevel) of this
                                // list (null: the instances first .. first + nlevel - 1)
  int max_m;                    // largest front in the level
  int max_pm;                   // largest p*m in the level
  int max_p;                    // largest p in the level
  int fault = -1;               // factorisation test hook: front instance whose first
                                // pivot column is zeroed on its fully summed rows after
                                // assembly (-1 = none)
};
// Subtree sweeps of the deep levels: one workgroup per subtree (a front at
// depth D with all its descendants), the update vectors between its fronts in
// LDS.  Every fused level must be one the wavefront kernels take (m <= 128,
// p <= 64).
struct FuseArgs {
  const int* lev = nullptr;     // per subtree: K + 1 offsets into fl (relative level j = depth - D)
  const int4* fl = nullptr;     // {front, its slot, child 0's slot, child 1's slot} (-1: none / root)
  int K = 0;                    // levels per subtree
  int ntrees = 0;               // subtrees (fronts at depth D)
  int slot_q = 0;               // largest summed q over a subtree's slots
  int max_m = 0, max_p = 0;     // over the fused levels
};
// Whether the subtree sweeps run these levels with nr right-hand sides (the
// wavefront kernels' limits and the LDS of the slots).
bool subtree_ok(const FuseArgs& z, size_t elem, int nr);
template <typename T>
void launch_fwd_subtree(hipStream_t st, const LevelArgs& a, const FuseArgs& z, const T* lpk, const int* piv,
                        T* vec, const RhsSet& r);
template <typename T>
void launch_bwd_subtree(hipStream_t st, const LevelArgs& a, const FuseArgs& z, const T* upk, T* vec, T* u,
                        const RhsSet& r);

// Launch shape of one level's kernel: kind 0 = the built-in rule for the
// level, else an explicit choice (the autotuner's).  Factorisation: kind 1 =
// one wavefront per front with the front in LDS (small fronts), kind 2 = the
// panel kernel with nb-column panels and ntf threads per front.
struct FactorShape {
  int kind = 0, nb = 0, ntf = 0;
};
// Sweeps: kind 1 = one wavefront per front (levels with m <= 128, p <= 64),
// kind 2 = `parts` workgroups of ntl threads per front; kp = operator terms
// per thread held in registers ahead of the right-hand side.
struct SweepShape {
  int kind = 0, kp = 0, ntl = 0, parts = 0;
};
// The built-in choices, whether a shape runs a level (instantiated variant,
// LDS, the kernels' own limits), and the shapes the autotuner times for a
// level (the built-in choice first).  elem = bytes per complex entry.
FactorShape factor_default(const LevelArgs& a, size_t elem);
bool factor_shape_ok(const LevelArgs& a, size_t elem, const FactorShape& s);
std::vector<FactorShape> factor_candidates(const LevelArgs& a, size_t elem);
SweepShape sweep_default(const LevelArgs& a, bool fwd, size_t elem);
bool sweep_shape_ok(const LevelArgs& a, bool fwd, size_t elem, int nr, const SweepShape& s);
std::vector<SweepShape> sweep_candidates(const LevelArgs& a, bool fwd, size_t elem, int nr);
// Assembly (original entries + extend-add of the children) and partial LU of
// every front of one level.  A shape that does not run the level is an
// STF_EINVAL error.
template <typename T>
void launch_front_factor(hipStream_t st, const LevelArgs& a, T* fac, T* lpk, T* upk, int* piv, int* flag,
                         double tau, FactorShape sh = {});
template <typename T>
void launch_sweep_fwd(hipStream_t st, const LevelArgs& a, const T* fac, const int* piv, T* vec,
                      const RhsSet& r, SweepShape sh = {});
template <typename T>
void launch_sweep_bwd(hipStream_t st, const LevelArgs& a, const T* upk, T* vec, T* u,
                      const RhsSet& r, SweepShape sh = {});
// z = sum_k P_k u_k for every problem of a set (ScatDev table of nprob entries,
// grid sized by the largest nx, ny), skipping problems with pact[p] == 0.
template <typename T>
void launch_scatter(hipStream_t st, const T* u, const SubDev* subs, const int4* cover_x,
                    const int4* cover_y, const ScatDev* probs, int nprob, int max_nx, int max_ny,
                    const int* pact, const RhsSet& r);

// Staged (multiplicative) order of the round: r_s = v_s - A z_s on the own
// boxes I_k of the scount subdomains slist[sfirst ..) (rbuf: slot s at
// rbuf + s * rstride), and z_s += sum over the stage of P_k u_k on their
// extended boxes (inst[k] != 0 marks the stage's subdomains; each node is
// added once, by its lowest covering member).  maxw x maxh bounds the boxes.
void launch_stage_residual(hipStream_t st, const double2* keps, const double2* gc,
                           const SubDev* subs, const ScatDev* probs, const int* slist, int sfirst,
                           int scount, int maxw, int maxh, const int* pact, const RhsSet& r,
                           double2* rbuf, long long rstride);
template <typename T>
void launch_stage_scatter(hipStream_t st, const T* u, const SubDev* subs, const ScatDev* probs,
                          const int4* cover_x, const int4* cover_y, const int* slist, int sfirst,
                          int scount, int maxw, int maxh, const int* inst, const int* pact,
                          const RhsSet& r);
// The first stage's sum written over every node of every problem (members by
// inst, as launch_stage_scatter adds them; 0 where none covers a node): no
// zero fill of z is needed before it.
template <typename T>
void launch_stage_scatter_first(hipStream_t st, const T* u, const SubDev* subs, const int4* cover_x,
                                const int4* cover_y, const ScatDev* probs, int nprob, int max_nx,
                                int max_ny, const int* inst, const int* pact, const RhsSet& r);
void launch_zero(hipStream_t st, double2* p, long long n);
// Eq. (20): per_sub[k] = |u_k| on Omega_k outside I_k (nsub subdomains), out[0] = their sum.
template <typename T>
void launch_overlap_norm(hipStream_t st, const T* u, const SubDev* subs, int nsub, double* per_sub,
                         double* out);

// Krylov (kernels_krylov.hip).  Vectors of n complex doubles; V holds nv vectors
// with leading dimension ld (elements).
int krylov_blocks(long long n);
// partial[blk][i] = V_i^H w per block (+ |w|^2 partials when norm_partial);
// gated kernels run only when *gate != 0 (gate may be null).
void launch_mdot(hipStream_t st, const double2* V, long long ld, int nv, const double2* w,
                 long long n, double2* partial, double* norm_partial, const int* gate);
// h[i] = sum_b partial[b * stride + i] for i < nv (stride 0 means nv).
void launch_mdot_reduce(hipStream_t st, const double2* partial, int nblk, int nv, double2* h,
                        const int* gate, int stride = 0);
// Register-resident Gram-Schmidt passes over bases of 1..32 vectors (one entry
// per thread, gs_blocks(n) workgroups; partials [blk][gs_stride(nv)]).
//   GS_DOT:        partial = V^H w, |w|^2 partials
//   GS_UPDATE_DOT: w -= V h, then partial = V^H w and |w|^2 of the new w
//   GS_UPDATE:     w -= V h, |w|^2 partials
//   GS_UPDATE_NORMALIZE: w -= V h, then vout = w / |w| with |w|^2 = nrm_in - |h|^2
//                  (stored to nrm_out; the pass after which w is orthogonal to V)
enum { GS_DOT = 0, GS_UPDATE_DOT = 1, GS_UPDATE = 2, GS_UPDATE_NORMALIZE = 3 };
int gs_blocks(long long n, int nv);   // workgroups of a pass over a basis of nv vectors
int gs_stride(int nv);    // 8, 16 or 32; 0 when nv > 32 (use launch_mdot / launch_mupdate)
void launch_gs(hipStream_t st, int mode, const double2* V, long long ld, int nv, const double2* h,
               double2* w, long long n, double2* partial, double* norm_partial, const int* gate,
               double2* vout = nullptr, const double* nrm_in = nullptr, double* nrm_out = nullptr);
// The same pass for nr (<= MAX_RHS) independent right-hand sides in one
// launch (blockIdx.y = s); every pointer of launch_gs per right-hand side,
// basis length nv, leading dimension ld and vector length n shared.
struct GsSet {
  const double2* V[MAX_RHS] = {};
  const double2* h[MAX_RHS] = {};
  double2* w[MAX_RHS] = {};
  double2* partial[MAX_RHS] = {};
  double* npart[MAX_RHS] = {};
  const int* gate[MAX_RHS] = {};
  double2* vout[MAX_RHS] = {};
  const double* nrm_in[MAX_RHS] = {};
  double* nrm_out[MAX_RHS] = {};
};
void launch_gs_set(hipStream_t st, int mode, int nr, const GsSet& S, long long ld, int nv, long long n);
// Between the passes: h[i] = sum_b partial[b * stride + i] (i < nv) and
// out = sum of the nblk norm partials, with ref also gate = (out < ref/2).
void launch_gs_reduce(hipStream_t st, const double2* partial, int nblk, int stride, int nv,
                      double2* h, const double* npart, double* out, const double* ref, int* gate);
struct GsRedSet {
  const double2* partial[MAX_RHS] = {};
  double2* h[MAX_RHS] = {};
  const double* npart[MAX_RHS] = {};
  double* out[MAX_RHS] = {};
  const double* ref[MAX_RHS] = {};
  int* gate[MAX_RHS] = {};
};
void launch_gs_reduce_set(hipStream_t st, int nr, const GsRedSet& S, int nblk, int stride, int nv);
// w -= V h (+ |w|^2 partials).
void launch_mupdate(hipStream_t st, const double2* V, long long ld, int nv, const double2* h,
                    double2* w, long long n, double* norm_partial, const int* gate);
// out = sum of partials; decide: gate = (out < ref/2).
void launch_norm_reduce(hipStream_t st, const double* partial, int n, double* out,
                        const double* ref, int* gate, int decide);
void launch_hacc(hipStream_t st, double2* h1, const double2* h2, int nv, const int* gate);
// v = w / sqrt(nrm2) (skipped when skip and skip[0] != 0)
void launch_scale(hipStream_t st, const double2* w, const double* nrm2, double2* v,
                  long long n, const int* skip = nullptr);
// The end of Arnoldi step j in one launch: Givens step j of FGMRES on device
// (H column-major, ldh = m+1; with gate[0] != 0 the column is h + h2 and |w|^2
// is wnorm2_alt[0], stored to wnorm2[0]) and v = w / |w| (skipped when
// gate[0] != 0).  |w|^2 and the residual estimate also go to host_out[0..1]
// (device-visible pinned host memory) when it is given.
void launch_scale_givens(hipStream_t st, const double2* w, double2* v, long long n, double2* H,
                         const double2* h, double* wnorm2, double* cs, double2* sn, double2* g,
                         int j, int ldh, double* est_out, const double2* h2, const int* gate,
                         const double* wnorm2_alt, double* host_out);
struct GivensSet {
  const double2* w[MAX_RHS] = {};
  double2* v[MAX_RHS] = {};
  double2* H[MAX_RHS] = {};
  const double2* h[MAX_RHS] = {};
  double* wnorm2[MAX_RHS] = {};
  double* cs[MAX_RHS] = {};
  double2* sn[MAX_RHS] = {};
  double2* g[MAX_RHS] = {};
  double* est[MAX_RHS] = {};
  const double2* h2[MAX_RHS] = {};
  const int* gate[MAX_RHS] = {};
  const double* wnorm2_alt[MAX_RHS] = {};
  double* host_out[MAX_RHS] = {};
};
void launch_scale_givens_set(hipStream_t st, int nr, const GivensSet& S, long long n, int j, int ldh);
// The end and start of FGMRES cycles for nr (<= MAX_RHS) right-hand sides in
// one launch each (blockIdx selects s): y_s = R_s^{-1} g_s over k_s columns
// (H, g, y, k), x_s += Z_s y_s (Z, k, y, x), v_s = r_s / sqrt(nrm2_s) with
// gs_s = (sqrt(nrm2_s), 0, ...) (r, nrm2, v, gs).
struct CycleSet {
  const double2* H[MAX_RHS] = {};
  const double2* g[MAX_RHS] = {};
  double2* y[MAX_RHS] = {};
  int k[MAX_RHS] = {};
  const double2* Z[MAX_RHS] = {};
  double2* x[MAX_RHS] = {};
  const double2* r[MAX_RHS] = {};
  const double* nrm2[MAX_RHS] = {};
  double2* v[MAX_RHS] = {};
  double2* gs[MAX_RHS] = {};
};
void launch_trisolve_set(hipStream_t st, int nr, const CycleSet& S, int ldh);
void launch_xupdate_set(hipStream_t st, int nr, const CycleSet& S, long long ld, long long n);
void launch_cycle_start_set(hipStream_t st, int nr, const CycleSet& S, long long n, int glen);
// y += x
void launch_axpy(hipStream_t st, double2* y, const double2* x, long long n);

// ---------------------------------------------------------------------------
// Batched FGMRES (kernels_batch.hip): every launch covers all systems; sc holds
// 16 doubles per system ([0] |b|^2, [2] |r|^2, [3] |w|^2, [4] estimate, [6] |w|^2
// before the first update, [8] |w|^2 after the second, [10] non-finite flag).
// ---------------------------------------------------------------------------
int bgs_class(int nv);    // chunk class of the Gram-Schmidt pass over nv vectors (-1: > 32)
void launch_bstencil(hipStream_t st, int mode, const double2* x, const double2* b, double2* y,
                     const double2* keps, const double2* gc, const SysDev* sys, const int* tsys,
                     int ntiles, const int* gate, double* partial);
void launch_bnorm2(hipStream_t st, const double2* v, const SysDev* sys, const int* bsys, int nblk,
                   double* npart);
void launch_bsum(hipStream_t st, const double* partial, const SysDev* sys, int nsys, int ci,
                 const int* gate, double* sc, int out);
void launch_bgs(hipStream_t st, int mode, const double2* V, long long ld, int nv, const double2* h,
                int hs, double2* w, const SysDev* sys, const int* bsys, int nblk, const int* act,
                const int* rgate, double* partial, double* npart, double2* vout, double* sc, int nin,
                int nout);
void launch_bgs_reduce(hipStream_t st, const double* partial, int nv, const SysDev* sys, int nsys,
                       const int* act, const int* rgate_in, double2* h, int hs, const double* npart,
                       double* sc, int out, int ref, int* rgate_out);
void launch_bgivens_scale(hipStream_t st, const double2* w, double2* v, const SysDev* sys,
                          const int* bsys, int nblk, int nsys, double2* H, const double2* h1,
                          const double2* h2, int m, double* sc, double* cs, double2* sn, double2* g,
                          int j, int* act, const int* rgate, int* kcol, int* it, double* hist,
                          int hcap, double tol, int max_iter);
void launch_bpact(hipStream_t st, const int* act, int nslot, int nprob, int* pact);
void launch_bcycle_start(hipStream_t st, const double2* r, double2* v, const SysDev* sys,
                         const int* bsys, int nblk, int nsys, const double* sc, double2* g, int glen,
                         int* act, int* cyc, int* kcol, const int* it, double tol, int max_iter);
void launch_btrisolve(hipStream_t st, const double2* H, int m, const double2* g, double2* y,
                      const int* kcol, const int* cyc, int nsys);
void launch_bxupdate(hipStream_t st, const double2* Z, long long ld, const double2* y, int hs,
                     double2* x, const SysDev* sys, const int* bsys, int nblk, const int* kcol,
                     const int* cyc);
void launch_bstatus(hipStream_t st, const double* sc, const int* it, const int* cyc, int nsys,
                    double* host_out);

// ---------------------------------------------------------------------------
// Learned warm start (kernels_nn.hip).  FP32 tensors, all on `st`.
// ---------------------------------------------------------------------------
// C[b] = alpha A[b] B[b] + beta C[b] with element strides (A: b, m, k; B: b, k, n; C: b, m, n).
void nn_gemm(hipStream_t st, int batch, int M, int N, int K, const float* A, long long sAb,
             long long sAm, long long sAk, const float* B, long long sBb, long long sBk,
             long long sBn, float* C, long long sCb, long long sCm, long long sCn, float alpha,
             float beta);
void nn_dft_y(hipStream_t st, const float* T, const float2* ey, int planes, int n, int M,
              bool grad_scale, float2* H);
// out (per plane, n x n) = alpha Ainv S + beta out with S the x inverse of G
// (as nn_dft_x_inv), in one pass per plane (n % 16 == 0, n <= 1024, M <= 22).
bool nn_spec_inv_ok(int n, int M);
void nn_spec_inv(hipStream_t st, const float2* G, const float2* ex, int planes, int n, int M,
                 bool weighted, const float* ainv, float alpha, float beta, float* out, long long npix);
void nn_dft_x_inv(hipStream_t st, const float2* G, const float2* ex, int planes, int n, int M,
                  bool weighted, float* S);
void nn_mix_fwd(hipStream_t st, const float2* H, const float* Rre, const float* Rim, int B, int W,
                int NM, float2* G);
void nn_mix_bwd(hipStream_t st, const float2* H, const float2* dG, const float* Rre,
                const float* Rim, int B, int W, int NM, float2* dH, float* dRre, float* dRim);
bool nn_width_supported(int cin, int w);
void nn_pw_fwd(hipStream_t st, int ci, int co, bool act, const float* in, const float* Wm,
               const float* bias, const float* add, long long npix, int B, float* pre, float* out);
// Inference of one layer of the compiled shape (n = 256, M = 16, width 16):
// out = act(W h + bias + alpha Ainv S) per plane, S the rows k_dft_x_inv wrote
// (4M x n per plane), without storing the spectral branch.
bool nn_spec_pw_ok(int n, int M, int W);
// The weighted x-inverse rows (4M x n per plane) of the compiled shape.
void nn_spec_rows(hipStream_t st, const float2* G, const float2* ex, int planes, int n, int M, float* S);
void nn_spec_pw(hipStream_t st, const float* S, const float* ainv, float alpha, const float* hin,
                const float* Wm, const float* bias, long long npix, int B, int n, int M, int W, bool act,
                float* out);
int nn_pw_bwd_blocks();
void nn_pw_bwd(hipStream_t st, int ci, int co, bool act, const float* dout, const float* pre,
               const float* in, const float* Wm, long long npix, int B, float* dpre, float* din,
               float* partial, float* grad_w);
int nn_loss_blocks();
void nn_loss(hipStream_t st, const float* y, const float* t, long long per, int B, double* partial,
             double* den, double* loss, float* dy);
// Adam on the FP32 master parameters p; q gets them rounded to BF16.
void nn_adam(hipStream_t st, float* p, const float* g, float* m, float* v, long long n, double lr,
             int step, double beta1, double beta2, double eps, float* q);
// q = p rounded to BF16 (round to nearest, ties to even), held as FP32 values.
void nn_quantize_bf16(hipStream_t st, const float* p, float* q, long long n);
void nn_features(hipStream_t st, const double2* keps, const double2* b, double k0sq, int nx,
                 int pml_x, int pml_y, const int2* org, int ntiles, int n, float* f);
void nn_fields(hipStream_t st, const double2* x, int nx, int pml_x, int pml_y, const int2* org,
               int ntiles, int n, float* t);
void nn_blend(hipStream_t st, const float* pred, const int* oy, int nty, const int* ox, int ntx,
              int n, int pml_x, int pml_y, int inx, int iny, int nx, int ny, double2* x0);

}  // namespace stf
