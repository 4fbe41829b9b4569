// Multifrontal LU of the subdomain operators (Sec. 2.4, Eq. (22)) and the
// front sweeps of the local solves (Eq. (23)), batched over every front of one
// elimination-tree level across all subdomains; T = double2 (complex128) or
// float2 (complex64).
//
// Storage: front f of order m = p + q is an m x m COLUMN-major block at
// fac_off, entry (r, c) at F[c*m + r], with the p separator (fully summed)
// variables first:  [F11 F12; F21 F22].  After factorisation F11 holds L11
// (unit lower, implicit 1) and U11, F12 holds U12, F21 holds L21 and F22 the
// Schur complement that the parent gathers by extend-add.  Column-major makes
// every step of the column-oriented triangular sweeps and every LU panel a
// contiguous, coalesced read.  Pivoting is partial, restricted to the p fully
// summed rows; swaps are applied to whole rows.  After the partial LU the row
// exchanges are stored as a gather permutation (piv[k] = source row of row k
// of P b) and every diagonal block (DIB x DIB) of L11 and of U11 is replaced by
// its inverse, so that each step of the triangular sweeps is a matrix-vector
// product (Eq. (23) applied as products, as the paper describes the solve
// phase) with no serial chain over the rows.
//
// Front vectors: each front owns m entries at vec_off.  The forward sweep
// leaves [y_p ; update contribution] there; in the backward sweep a front
// reads y_p and the x_q that its parent put in place of the update
// contribution, and puts its own [x_p ; x_q] into the update parts of its
// children.  Every write has one owner, so the sweeps are deterministic
// without atomics.
//
// Two team sizes: fronts of a level whose largest order fits a wavefront are
// handled one per 64-lane workgroup with no workgroup barriers (lane = row);
// larger fronts get a 256-thread workgroup each.
#include <algorithm>

#include "cplx.h"
#include "stf_internal.h"

namespace stf {

namespace {

constexpr int NT = 256;        // threads of a large-front workgroup
constexpr int UC = 32;         // columns of U staged in LDS per trailing-update chunk
constexpr int DIB = 64;        // inverted diagonal blocks of L11 and U11
constexpr int CR = 32;         // rows (or columns) staged per chunk by the inversion tail
// Leading dimension of the inversion tail's diagonal blocks for a level whose
// separators are at most max_p wide.
__host__ __device__ constexpr int inv_ld(int max_p) { return max_p <= 32 ? 32 : DIB; }

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Packed sweep operators of a front of order m with p separator variables:
//   forward:  column k < p holds rows k+1 .. m-1 of [L11^{-1}; M'] (the unit
//             diagonal is implicit), column after column;
//   backward: column c holds rows 0 .. min(c, p-1) of [U11^{-1}  V'].
// Only the entries the sweeps read are stored, each column contiguous.
__host__ __device__ inline int lpk_col(int m, int k) { return k * (m - 1) - k * (k - 1) / 2; }
__host__ __device__ inline int upk_col(int p, int c) {
  return c < p ? c * (c + 1) / 2 : p * (p + 1) / 2 + (c - p) * p;
}
// Element offsets of row r, column k in the packed forms.
struct LowerAt {
  int m, r;
  __device__ int operator()(int k) const { return lpk_col(m, k) + r - k - 1; }
};
struct UpperAt {
  int p, r;
  __device__ int operator()(int c) const { return upk_col(p, c) + r; }
};

// Coefficient of local row `node` towards direction `dir` (0 = diagonal).
__device__ inline double2 local_coef(const LevelArgs& a, const SubDev& s, int node, int dir) {
  int tx = node % s.nxl, ty = node / s.nxl;
  const double2* cx = a.lcoef + s.cx_off;   // (w, e) pairs per local column
  const double2* cy = a.lcoef + s.cy_off;   // (w, e) pairs per local row
  double2 xw = cx[2 * tx], xe = cx[2 * tx + 1], yw = cy[2 * ty], ye = cy[2 * ty + 1];
  switch (dir) {
    case 1: return xw;
    case 2: return xe;
    case 3: return yw;
    case 4: return ye;
    default: {
      double2 ke = a.keps[s.gbase + (long long)(s.oy0 + ty) * s.gnx + (s.ox0 + tx)];
      return make_double2(ke.x - ((xw.x + xe.x) + (yw.x + ye.x)),
                          ke.y - ((xw.y + xe.y) + (yw.y + ye.y)));
    }
  }
}

// Assembly of one front into a column-major buffer G with leading dimension m
// (global memory or LDS): zero, original entries, then the children's Schur
// complements one child at a time.  `sync` separates the phases.
template <typename T, typename Sync>
__device__ inline void assemble_front(const LevelArgs& a, const T* __restrict__ fac,
                                      const FrontDev& f, T* G, int tid, int nthr, Sync sync) {
  const int m = f.p + f.q;
  const long long mm = (long long)m * m;
  for (long long t = tid; t < mm; t += nthr) G[t] = czero<T>();
  sync();
  const SubDev s = a.subs[f.sub];
  for (int t = tid; t < f.ent_cnt; t += nthr) {
    SymEntry e = a.ents[f.ent_off + t];
    int r = e.rc & 0xffff, c = (e.rc >> 16) & 0xffff;
    G[(long long)c * m + r] = from_d2<T>(local_coef(a, s, e.nd >> 3, e.nd & 7));
  }
  sync();
  // Extend-add: the child map is injective, so the entries of one child go to
  // distinct places and a thread takes UB of them per round trip (all loads of
  // the batch, then all read-modify-writes).
  constexpr int UB = 8;
  for (int ci = 0; ci < f.nchild; ++ci) {
    const FrontDev cf = a.fronts[a.children[f.child_off + ci]];
    const int mc = cf.p + cf.q, q = cf.q;
    const T* S = fac + cf.fac_off + (long long)cf.p * mc + cf.p;   // F22 of the child
    const int* cm = a.cmap + cf.cmap_off;
    const int qq = q * q;
    for (int t0 = tid; t0 < qq; t0 += nthr * UB) {
      T v[UB];
      long long d[UB];
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        const int t = t0 + u * nthr;
        const int j = t / q, i = t - j * q;                          // (i, j) of S, i fastest
        const bool ok = t < qq;
        v[u] = ok ? S[(long long)j * mc + i] : czero<T>();
        d[u] = ok ? (long long)cm[j] * m + cm[i] : -1;
      }
      T g[UB];
#pragma unroll
      for (int u = 0; u < UB; ++u) g[u] = d[u] >= 0 ? G[d[u]] : czero<T>();
#pragma unroll
      for (int u = 0; u < UB; ++u)
        if (d[u] >= 0) G[d[u]] = cadd(g[u], v[u]);
    }
    sync();
  }
}

// The same front assembled in one pass, for fronts in global memory: every
// entry of G is written once, as the sum of the children's Schur complements
// that map to it (through inverse child maps kept in LDS, icm: 2 m ints), and
// the original entries are added after.  No zero fill and no read-modify-write
// of G by the extend-add.  The sum is taken in the order child 0, child 1,
// original entry.
template <typename T>
__device__ inline void assemble_front_gather(const LevelArgs& a, const T* __restrict__ fac,
                                             const FrontDev& f, T* __restrict__ G, int tid,
                                             int nthr, int* icm) {
  const int m = f.p + f.q;
  for (int t = tid; t < 2 * m; t += nthr) icm[t] = -1;
  __syncthreads();
  const T* S[2] = {fac, fac};                                        // F22 of the children
  int ld[2] = {0, 0};
#pragma unroll
  for (int ci = 0; ci < 2; ++ci) {
    if (ci < f.nchild) {
      const FrontDev cf = a.fronts[a.children[f.child_off + ci]];
      const int mc = cf.p + cf.q;
      S[ci] = fac + cf.fac_off + (long long)cf.p * mc + cf.p;
      ld[ci] = mc;
      const int* cm = a.cmap + cf.cmap_off;
      for (int i = tid; i < cf.q; i += nthr) icm[ci * m + cm[i]] = i;
    }
  }
  __syncthreads();
  constexpr int UB = 8;
  const int mm = m * m;                                              // m <= 46340
  for (int t0 = tid; t0 < mm; t0 += nthr * UB) {
    T v0[UB], v1[UB];
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      const int t = t0 + u * nthr;
      const int c = t / m, r = t - c * m;                            // r fastest
      const bool ok = t < mm;
      const int r0 = ok ? icm[r] : -1, c0 = ok ? icm[c] : -1;
      const int r1 = ok ? icm[m + r] : -1, c1 = ok ? icm[m + c] : -1;
      v0[u] = (r0 >= 0 && c0 >= 0) ? S[0][(long long)c0 * ld[0] + r0] : czero<T>();
      v1[u] = (r1 >= 0 && c1 >= 0) ? S[1][(long long)c1 * ld[1] + r1] : czero<T>();
    }
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      const int t = t0 + u * nthr;
      if (t < mm) G[t] = cadd(v0[u], v1[u]);
    }
  }
  __syncthreads();
  const SubDev s = a.subs[f.sub];
  for (int t = tid; t < f.ent_cnt; t += nthr) {
    SymEntry e = a.ents[f.ent_off + t];
    int r = e.rc & 0xffff, c = (e.rc >> 16) & 0xffff;
    const long long idx = (long long)c * m + r;
    G[idx] = cadd(G[idx], from_d2<T>(local_coef(a, s, e.nd >> 3, e.nd & 7)));
  }
  __syncthreads();
}

// Pivot choice for column k over rows [k, pend) with amax over [k, nrow) of a
// column-major column `col`; one wavefront, result in every lane.
template <typename T>
__device__ inline void wave_pivot(const T* col, int k, int pend, int nrow, int lane, int& bi,
                                  typename RealOf<T>::type& best, typename RealOf<T>::type& amax) {
  using R = typename RealOf<T>::type;
  best = (R)-1;
  amax = (R)0;
  bi = k;
  for (int r = k + lane; r < nrow; r += 64) {
    R v = cabs2(col[r]);
    amax = v > amax ? v : amax;
    if (r < pend && v > best) { best = v; bi = r; }
  }
  for (int o = 32; o > 0; o >>= 1) {
    R ob = __shfl_xor(best, o, 64);
    int oi = __shfl_xor(bi, o, 64);
    R oa = __shfl_xor(amax, o, 64);
    if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    amax = oa > amax ? oa : amax;
  }
}

// Static perturbation of a tiny pivot: |pivot| < tau * max |column| (or zero).
template <typename T>
__device__ inline bool perturb(T& v, typename RealOf<T>::type best, typename RealOf<T>::type amax,
                               double tau) {
  using R = typename RealOf<T>::type;
  R thr = (R)tau * sqrt(amax);
  if (sqrt(best) > thr && best > (R)0) return false;
  R mag = sqrt(cabs2(v));
  R tgt = thr > (R)0 ? thr : (R)1e-30;
  v = mag > (R)0 ? T{v.x / mag * tgt, v.y / mag * tgt} : T{tgt, (R)0};
  return true;
}

// Row exchanges ip[k] (LAPACK order) -> gather permutation stored back in ip:
// (P b)[k] = b[ip[k]].  tmp: p ints.  One thread.
__device__ inline void pivots_to_perm(int* ip, int* tmp, int p) {
  for (int k = 0; k < p; ++k) tmp[k] = k;
  for (int k = 0; k < p; ++k) {
    int r2 = ip[k];
    int t = tmp[k]; tmp[k] = tmp[r2]; tmp[r2] = t;
  }
  for (int k = 0; k < p; ++k) ip[k] = tmp[k];
}

// In-place inverse of the unit lower triangle of the n x n column-major block
// G (ld): column j of the inverse is -(L[:, j] + X[:, j+1:] L[j+1:, j]) below
// the diagonal, built from the right.  One wavefront (n <= 64); col: n entries.
template <typename T>
__device__ inline void invert_lower_unit(T* G, int ld, int n, T* col, int lane) {
  for (int j = n - 2; j >= 0; --j) {
    col[lane] = (lane > j && lane < n) ? G[j * ld + lane] : czero<T>();
    wave_sync();
    if (lane > j && lane < n) {
      T x = col[lane];
      for (int k = j + 1; k < lane; ++k) x = cfma(G[k * ld + lane], col[k], x);
      G[j * ld + lane] = T{-x.x, -x.y};
    }
    wave_sync();
  }
}

// In-place inverse of the upper triangle (diagonal included) of the n x n
// column-major block G: X[j][j] = 1/U[j][j], X[0:j, j] = -X[0:j, 0:j] U[0:j, j] / U[j][j],
// built from the left.  One wavefront (n <= 64); col: n entries.
template <typename T>
__device__ inline void invert_upper(T* G, int ld, int n, T* col, int lane) {
  using R = typename RealOf<T>::type;
  for (int j = 0; j < n; ++j) {
    col[lane] = (lane <= j) ? G[j * ld + lane] : czero<T>();
    wave_sync();
    const T dinv = cdiv(T{(R)1, (R)0}, col[j]);
    if (lane < j) {
      T x = czero<T>();
      for (int k = lane; k < j; ++k) x = cfma(G[k * ld + lane], col[k], x);
      x = cmul(x, dinv);
      G[j * ld + lane] = T{-x.x, -x.y};
    } else if (lane == j) {
      G[j * ld + j] = dinv;
    }
    wave_sync();
  }
}

// ---------------------------------------------------------------------------
// Factorisation, small fronts: one wavefront per front, front in LDS.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(64) void k_factor_small(LevelArgs a, T* __restrict__ fac,
                                                     T* __restrict__ lpk, T* __restrict__ upk,
                                                     int* __restrict__ piv,
                                                     int* __restrict__ flag, double tau) {
  using R = typename RealOf<T>::type;
  extern __shared__ unsigned char smem_raw[];
  T* G = reinterpret_cast<T*>(smem_raw);
  const FrontDev f = a.fronts[a.first + blockIdx.x];
  const int m = f.p + f.q, p = f.p, lane = threadIdx.x;
  assemble_front<T>(a, fac, f, G, lane, 64, [] { wave_sync(); });
  if (a.first + (int)blockIdx.x == a.fault) {         // planted fault (test hook)
    for (int r = lane; r < p; r += 64) G[r] = czero<T>();
    wave_sync();
  }
  int* ip = piv + f.piv_off;
  // Pivot choice, perturbation and row exchange of step k (column k as it
  // stands), then the multipliers of column k.
  auto pivot_step = [&](int k) {
    int bi;
    R best, amax;
    wave_pivot(G + k * m, k, p, m, lane, bi, best, amax);
    if (lane == 0) {
      T v = G[k * m + bi];
      if (perturb(v, best, amax, tau)) {
        G[k * m + bi] = v;
        atomicOr(flag, 1);
      }
      ip[k] = bi;
    }
    wave_sync();
    if (bi != k)
      for (int c = lane; c < m; c += 64) {
        T t0 = G[c * m + k];
        G[c * m + k] = G[c * m + bi];
        G[c * m + bi] = t0;
      }
    wave_sync();
    const T dinv = cdiv(T{(R)1, (R)0}, G[k * m + k]);
    for (int r = k + 1 + lane; r < m; r += 64) G[k * m + r] = cmul(G[k * m + r], dinv);
    wave_sync();
  };
  // Steps are taken in pairs (k, k+1): after step k only column k+1 is
  // updated, so that step k+1 can choose its pivot; the rest of the trailing
  // block then takes one rank-2 update, read and written once per pair.
  int k = 0;
  for (; k + 1 < p; k += 2) {
    pivot_step(k);
    for (int r = k + 1 + lane; r < m; r += 64)
      G[(k + 1) * m + r] = cfms(G[k * m + r], G[(k + 1) * m + k], G[(k + 1) * m + r]);
    wave_sync();
    pivot_step(k + 1);
    // Row k+1 past column k+1 still lacks step k's update: u2 = row k+1 - l u1,
    // formed once (a lane per column) before the rank-2 update reads it.
    const T lk1 = G[k * m + k + 1];
    for (int c = k + 2 + lane; c < m; c += 64) G[c * m + k + 1] = cfms(lk1, G[c * m + k], G[c * m + k + 1]);
    wave_sync();
    for (int r = k + 2 + lane; r < m; r += 64) {
      const T l1 = G[k * m + r], l2 = G[(k + 1) * m + r];
      // four columns per round trip: all reads of a batch before its writes
      constexpr int CB = 4;
      for (int c0 = k + 2; c0 < m; c0 += CB) {
        T u1[CB], u2[CB], x[CB];
#pragma unroll
        for (int e = 0; e < CB; ++e) {
          const T* gc = G + min(c0 + e, m - 1) * m;
          u1[e] = gc[k];
          u2[e] = gc[k + 1];
          x[e] = gc[r];
        }
#pragma unroll
        for (int e = 0; e < CB; ++e)
          if (c0 + e < m) G[(c0 + e) * m + r] = cfms(l2, u2[e], cfms(l1, u1[e], x[e]));
      }
    }
    wave_sync();
  }
  if (k < p) {                      // odd p: a last single step
    pivot_step(k);
    for (int r = k + 1 + lane; r < m; r += 64) {
      const T l = G[k * m + r];
      for (int c = k + 1; c < m; ++c) G[c * m + r] = cfms(l, G[c * m + k], G[c * m + r]);
    }
    wave_sync();
  }
  T* colbuf = G + (long long)m * m;
  if (lane == 0) pivots_to_perm(ip, reinterpret_cast<int*>(colbuf + 64), p);
  wave_sync();
  if (p <= 32) {
    // Both triangles in one loop of p steps: lanes 0..31 build L11^{-1} by
    // columns from the right (lane = row), lanes 32..63 build U11^{-1} by rows
    // from the bottom (lane - 32 = column):
    //   X_L[r][j] = -(L[r][j] + sum_{j<k<r} X_L[r][k] L[k][j]),
    //   X_U[i][i] = 1/U[i][i],  X_U[i][c] = -X_U[i][i] sum_{i<k<=c} U[i][k] X_U[k][c].
    // The column of L (resp. row of U) a step needs is staged in colbuf first.
    // Both halves run the same instructions: x = init + sum_k a[k sa] b[k],
    // with per-lane pointers, strides and ranges (no divergent branches).
    const bool lo = lane < 32;
    const int cl = lo ? lane : lane - 32;
    for (int t = 0; t < p; ++t) {
      const int j = p - 2 - t, ii = p - 1 - t;
      const bool act = lo ? (j >= 0 && cl > j && cl < p) : (cl >= ii && cl < p);
      colbuf[lane] = act ? (lo ? G[j * m + cl] : G[cl * m + ii]) : czero<T>();
      wave_sync();
      const T dinv = cdiv(T{(R)1, (R)0}, colbuf[32 + ii]);
      const T* a = lo ? G + cl : colbuf + 32;              // L: X_L[cl][k]; U: U[ii][k]
      const T* b = lo ? colbuf : G + cl * m;               // L: L[k][j];    U: X_U[k][cl]
      const int sa = lo ? m : 1;
      const int k0 = lo ? j + 1 : ii + 1, k1 = lo ? cl : cl + 1;
      T x = lo ? colbuf[cl] : czero<T>();
      if (act)
        for (int k = k0; k < k1; ++k) x = cfma(a[k * sa], b[k], x);
      if (!lo) x = (cl == ii) ? T{-dinv.x, -dinv.y} : cmul(x, dinv);
      if (act) G[lo ? j * m + cl : cl * m + ii] = T{-x.x, -x.y};
      wave_sync();
    }
  } else {
    invert_lower_unit(G, m, p, colbuf, lane);
    invert_upper(G, m, p, colbuf, lane);
    wave_sync();
  }
  // M' = -L21 L11^{-1} and V' = -U11^{-1} U12, one entry per lane at a time over
  // the whole wavefront, written straight into the packed operators (G keeps
  // L21 and U12, which the products read).
  const int q = m - p;
  T* Lp = lpk + f.lpk_off;
  T* Up = upk + f.upk_off;
  for (int t = lane; t < q * p; t += 64) {
    const int j = t / q, r = p + (t - j * q);
    T acc = G[j * m + r];
    for (int k = j + 1; k < p; ++k) acc = cfma(G[k * m + r], G[j * m + k], acc);
    Lp[lpk_col(m, j) + r - j - 1] = T{-acc.x, -acc.y};
  }
  for (int t = lane; t < q * p; t += 64) {
    const int c = p + t / p, r = t - (c - p) * p;
    T acc = czero<T>();
    for (int k = r; k < p; ++k) acc = cfma(G[k * m + r], G[c * m + k], acc);
    Up[upk_col(p, c) + r] = T{-acc.x, -acc.y};
  }
  // Only the Schur complement F22 goes back to the front storage (the parent's
  // extend-add reads it).
  T* F = fac + f.fac_off;
  for (int t = lane; t < q * q; t += 64) {
    const int c = p + t / q, r = p + t % q;
    F[(long long)c * m + r] = G[c * m + r];
  }
  // The L11^{-1} and U11^{-1} parts of the packed operators.
  for (int k = 0; k < p; ++k)
    for (int r = k + 1 + lane; r < p; r += 64) Lp[lpk_col(m, k) + r - k - 1] = G[k * m + r];
  for (int c = 0; c < p; ++c)
    for (int r = lane; r <= c; r += 64) Up[upk_col(p, c) + r] = G[c * m + r];
}

// 16 x 16 x 4 matrix-core products (D = A B + C) in the precision of the front.
// Lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]; output element (i, j)
// of the 16 x 16 tile sits in lane j + 16 (i / 4), register i % 4 for FP32 and in
// lane j + 16 (i % 4), register i / 4 for FP64.
template <typename T> struct Mma;
template <> struct Mma<float2> {
  typedef float R;
  typedef float V __attribute__((ext_vector_type(4)));
  static __device__ inline V mma(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int l, int v) { return 4 * (l >> 4) + v; }
};
template <> struct Mma<double2> {
  typedef double R;
  typedef double V __attribute__((ext_vector_type(4)));
  static __device__ inline V mma(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int l, int v) { return (l >> 4) + 4 * v; }
};

// D = -A B over 16 x 16 complex tiles on the matrix cores, the tiles dealt to
// the nw wavefronts of the workgroup: rows [0, R), columns [0, C), inner index
// [0, K).  a(r, k) and b(k, c) return the operands (zero outside the triangle
// they describe); st(r, c, v) stores one result.
template <typename T, typename FA, typename FB, typename FS>
__device__ inline void mma_neg_product(int R, int C, int K, FA a, FB b, FS st, int wv, int nw,
                                       int lane) {
  using M = Mma<T>;
  using MR = typename M::R;
  const int l16 = lane & 15, lk = lane >> 4;
  const int ntr = (R + 15) / 16, ntc = (C + 15) / 16;
  for (int tt = wv; tt < ntr * ntc; tt += nw) {
    const int rb = 16 * (tt / ntc), cb = 16 * (tt % ntc);
    typename M::V accr = {0, 0, 0, 0}, acci = {0, 0, 0, 0};
    const int ra = rb + l16, cc = cb + l16;
    for (int k0 = 0; k0 < K; k0 += 4) {
      const int kk = k0 + lk;
      const T av = (ra < R && kk < K) ? a(ra, kk) : czero<T>();
      const T bv = (cc < C && kk < K) ? b(kk, cc) : czero<T>();
      accr = M::mma((MR)av.x, (MR)bv.x, accr);
      accr = M::mma((MR)-av.y, (MR)bv.y, accr);
      acci = M::mma((MR)av.x, (MR)bv.y, acci);
      acci = M::mma((MR)av.y, (MR)bv.x, acci);
    }
    if (cc < C) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = rb + M::row(lane, v);
        if (r < R) st(r, cc, T{-accr[v], -acci[v]});
      }
    }
  }
}

// One step of folding the per-block sweep operators of a large separator into
// full ones, on the columns [c0, c1) (at most DIB) of F, by the phase of the
// diagonal block [k0, k1) (its inverse on the diagonal, M' below, N' above):
//   LOWER: rows r >= k0:  X_r <- X_r + sum_{k0 <= k < min(k1, r)} F[r,k] X_k
//   UPPER: rows r < k1:   X_r <- [r < k0] X_r + sum_{max(k0, r) <= k < k1} F[r,k] X_k
// where X = F[:, c0:c1) and X_k (k in the block) is read from a copy staged in
// LDS (Xs, DIB x DIB) before any write.  Begins with a workgroup barrier.
template <typename T, bool LOWER, int NTF>
__device__ void fold_step(T* __restrict__ F, int m, int k0, int k1, int c0, int c1, T* Xs,
                          int tid) {
  constexpr int CC = 8;                       // columns per work item
  const int w = c1 - c0, wk = k1 - k0;
  __syncthreads();
  for (int t = tid; t < wk * w; t += NTF) {
    int c = t / wk, k = t - c * wk;
    Xs[k * DIB + c] = F[(long long)(c0 + c) * m + k0 + k];
  }
  __syncthreads();
  const int rlo = LOWER ? k0 : 0, rhi = LOWER ? m : k1;
  const int R = rhi - rlo, nch = (w + CC - 1) / CC;
  for (int t = tid; t < R * nch; t += NTF) {
    const int ch = t / R, r = rlo + (t - ch * R), cb = ch * CC;
    T acc[CC];
#pragma unroll
    for (int u = 0; u < CC; ++u)
      acc[u] = (cb + u < w && (LOWER || r < k0)) ? F[(long long)(c0 + cb + u) * m + r] : czero<T>();
    const int klo = LOWER ? k0 : max(k0, r), khi = LOWER ? min(k1, r) : k1;
#pragma unroll 4
    for (int k = klo; k < khi; ++k) {
      const T av = F[(long long)k * m + r];
      const T* xs = Xs + (k - k0) * DIB + cb;
#pragma unroll
      for (int u = 0; u < CC; ++u) acc[u] = cfma(av, xs[u], acc[u]);
    }
#pragma unroll
    for (int u = 0; u < CC; ++u)
      if (cb + u < w) F[(long long)(c0 + cb + u) * m + r] = acc[u];
  }
}

// ---------------------------------------------------------------------------
// Factorisation, large fronts: one workgroup of NTF threads per front (256, or
// 1024 for levels with at most one front per CU).  Assembly in
// global memory, then blocked right-looking LU: a panel of NB columns is
// factored in LDS by one wavefront, U12 is solved one column per thread and
// the trailing matrix is updated with each thread owning one row (its NB
// multipliers in registers) against U columns staged in LDS.
// ---------------------------------------------------------------------------
template <typename T, int NB, int NTF>
__global__ __launch_bounds__(NTF) void k_factor_large(LevelArgs a, T* __restrict__ fac,
                                                     T* __restrict__ lpk, T* __restrict__ upk,
                                                     int* __restrict__ piv,
                                                     int* __restrict__ flag, double tau) {
  using R = typename RealOf<T>::type;
  extern __shared__ unsigned char smem_raw[];
  T* P = reinterpret_cast<T*>(smem_raw);           // panel, column-major, ld = ldp
  __shared__ T Us[UC][NB + 1];                      // staged U columns
  __shared__ int s_piv[NB];
  __shared__ R s_best[NTF / 64], s_amax[NTF / 64];
  __shared__ int s_bi[NTF / 64];
  const FrontDev f = a.fronts[a.first + blockIdx.x];
  const int m = f.p + f.q, p = f.p, ldp = a.max_m;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  T* F = fac + f.fac_off;
  // The inverse child maps use the panel's LDS (2 max_m ints <= max_m NB T).
  assemble_front_gather<T>(a, fac, f, F, tid, NTF, reinterpret_cast<int*>(smem_raw));
  if (a.first + (int)blockIdx.x == a.fault) {         // planted fault (test hook)
    for (int r = tid; r < p; r += NTF) F[r] = czero<T>();
    __syncthreads();
  }
  int* ip = piv + f.piv_off;

  for (int kb = 0; kb < p; kb += NB) {
    const int nb = min(NB, p - kb);
    const int nr = m - kb;
    for (int t = tid; t < nb * nr; t += NTF) {
      int k = t / nr, r = t - k * nr;
      P[k * ldp + r] = F[(long long)(kb + k) * m + kb + r];
    }
    __syncthreads();
    // Panel LU: the pivot search on the first NPV threads (reduced per
    // wavefront and combined in LDS: largest |.|^2, ties to the lower row, as a
    // single wavefront would choose), the row updates on all NTF threads.
    constexpr int NPV = NTF < 256 ? NTF : 256;
    for (int k = 0; k < nb; ++k) {
      T* col = P + k * ldp;
      R best = (R)-1, amax = (R)0;
      int bi = k;
      for (int r = k + tid; tid < NPV && r < nr; r += NPV) {
        const R v = cabs2(col[r]);
        amax = v > amax ? v : amax;
        if (r < p - kb && v > best) {
          best = v;
          bi = r;
        }
      }
      for (int o = 32; o > 0; o >>= 1) {
        const R ob = __shfl_xor(best, o, 64);
        const int oi = __shfl_xor(bi, o, 64);
        const R oa = __shfl_xor(amax, o, 64);
        if (ob > best || (ob == best && oi < bi)) {
          best = ob;
          bi = oi;
        }
        amax = oa > amax ? oa : amax;
      }
      if (lane == 0 && tid < NPV) {
        s_best[wv] = best;
        s_amax[wv] = amax;
        s_bi[wv] = bi;
      }
      __syncthreads();
      if (tid == 0) {
        for (int w = 1; w < NPV / 64; ++w) {
          if (s_best[w] > best || (s_best[w] == best && s_bi[w] < bi)) {
            best = s_best[w];
            bi = s_bi[w];
          }
          amax = s_amax[w] > amax ? s_amax[w] : amax;
        }
        T v = col[bi];
        if (perturb(v, best, amax, tau)) {
          col[bi] = v;
          atomicOr(flag, 1);
        }
        s_piv[k] = bi;
        ip[kb + k] = kb + bi;
      }
      __syncthreads();
      bi = s_piv[k];
      if (bi != k && tid < nb) {
        T t0 = P[tid * ldp + k];
        P[tid * ldp + k] = P[tid * ldp + bi];
        P[tid * ldp + bi] = t0;
      }
      __syncthreads();
      const T dinv = cdiv(T{(R)1, (R)0}, col[k]);
      for (int r = k + 1 + tid; r < nr; r += NTF) {
        T l = cmul(col[r], dinv);
        col[r] = l;
        for (int c = k + 1; c < nb; ++c) P[c * ldp + r] = cfms(l, P[c * ldp + k], P[c * ldp + r]);
      }
      __syncthreads();
    }
    __syncthreads();
    for (int t = tid; t < nb * nr; t += NTF) {
      int k = t / nr, r = t - k * nr;
      F[(long long)(kb + k) * m + kb + r] = P[k * ldp + r];
    }
    // Row exchanges in the columns outside the panel, in pivot order, one
    // column per thread.
    for (int c = tid; c < m; c += NTF) {
      if (c >= kb && c < kb + nb) continue;
      T* Fc = F + (long long)c * m;
      for (int k = 0; k < nb; ++k) {
        int r2 = kb + s_piv[k];
        if (r2 != kb + k) {
          T t0 = Fc[kb + k];
          Fc[kb + k] = Fc[r2];
          Fc[r2] = t0;
        }
      }
    }
    __syncthreads();
    // U12 block row: L_d^{-1} F[kb:kb+nb, c] for every column c >= kb+nb.
    for (int c = kb + nb + tid; c < m; c += NTF) {
      T* Fc = F + (long long)c * m + kb;
      T x[NB];
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        if (i < nb) {
          T v = Fc[i];
#pragma unroll
          for (int t = 0; t < NB; ++t)
            if (t < i) v = cfms(P[t * ldp + i], x[t], v);
          x[i] = v;
          Fc[i] = v;
        }
      }
    }
    __syncthreads();
    // Trailing update F22 -= L21 U12 over rows/cols n0 .. m-1 on the matrix
    // cores: 16 x 16 complex tiles of F22, one wavefront per tile, the
    // multipliers from the LDS panel and U12 staged in LDS UC columns at a
    // time; four real products per complex K-step of four.
    const int n0 = kb + nb;
    const int R = m - n0;
    if (R > 0 && R < 128) {
      // Small trailing blocks: (row, column group) threads over the whole
      // workgroup, read-modify-writes in batches of TB columns.
      constexpr int TB = 8;
      const int G = NTF / R, g = tid / R, rr = tid - g * R;
      const int r = n0 + rr;
      const T* Pr = P + (r - kb);
      for (int c0 = n0; c0 < m; c0 += UC) {
        const int cw = min(UC, m - c0);
        __syncthreads();
        for (int t = tid; t < cw * NB; t += NTF) {
          int c = t / NB, k = t - c * NB;
          Us[c][k] = (k < nb) ? F[(long long)(c0 + c) * m + kb + k] : czero<T>();
        }
        __syncthreads();
        if (g < G) {
          for (int cb = g; cb < cw; cb += G * TB) {
            T acc[TB];
#pragma unroll
            for (int u = 0; u < TB; ++u) {
              const int c = cb + G * u;
              acc[u] = c < cw ? F[(long long)(c0 + c) * m + r] : czero<T>();
            }
            for (int t = 0; t < nb; ++t) {
              const T l = Pr[t * ldp];
#pragma unroll
              for (int u = 0; u < TB; ++u) acc[u] = cfms(l, Us[min(cb + G * u, UC - 1)][t], acc[u]);
            }
#pragma unroll
            for (int u = 0; u < TB; ++u) {
              const int c = cb + G * u;
              if (c < cw) F[(long long)(c0 + c) * m + r] = acc[u];
            }
          }
        }
      }
    } else if (R > 0) {
      using M = Mma<T>;
      using MR = typename M::R;
      const int l16 = lane & 15, lk = lane >> 4;
      const int ntr = (R + 15) / 16;
      for (int c0 = n0; c0 < m; c0 += UC) {
        const int cw = min(UC, m - c0);
        __syncthreads();
        for (int t = tid; t < cw * NB; t += NTF) {
          int c = t / NB, k = t - c * NB;
          Us[c][k] = (k < nb) ? F[(long long)(c0 + c) * m + kb + k] : czero<T>();
        }
        __syncthreads();
        const int ntc = (cw + 15) / 16, nt = ntr * ntc;
        // TU tiles per wavefront at a time: the loads of their F22 entries are
        // issued together before the products, so that the memory round trips
        // of the read-modify-writes overlap instead of following each other.
        constexpr int TU = (NTF >= 1024 || NB <= 8) ? 2 : 4, NWV = NTF / 64;
        for (int t0 = wv; t0 < nt; t0 += TU * NWV) {
          T cv[TU][4];
#pragma unroll
          for (int u = 0; u < TU; ++u) {
            const int tt = t0 + u * NWV;
            const int rb = n0 + 16 * (tt / ntc), cbb = 16 * (tt % ntc) + l16;
            const T* Fc = F + (long long)(c0 + cbb) * m;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int r = rb + M::row(lane, v);
              cv[u][v] = (tt < nt && cbb < cw && r < m) ? Fc[r] : czero<T>();
            }
          }
#pragma unroll
          for (int u = 0; u < TU; ++u) {
            const int tt = t0 + u * NWV;
            if (tt >= nt) break;
            const int rb = n0 + 16 * (tt / ntc), cb = 16 * (tt % ntc);
            typename M::V accr = {0, 0, 0, 0}, acci = {0, 0, 0, 0};
            const int ra = rb + l16, cbb = cb + l16;
            for (int k0 = 0; k0 < nb; k0 += 4) {
              const int kk = k0 + lk;
              const T av = (kk < nb && ra < m) ? P[kk * ldp + (ra - kb)] : czero<T>();
              const T bv = (kk < nb && cbb < cw) ? Us[cbb][kk] : czero<T>();
              accr = M::mma((MR)av.x, (MR)bv.x, accr);
              accr = M::mma((MR)-av.y, (MR)bv.y, accr);
              acci = M::mma((MR)av.x, (MR)bv.y, acci);
              acci = M::mma((MR)av.y, (MR)bv.x, acci);
            }
            if (cbb < cw) {
              T* Fc = F + (long long)(c0 + cbb) * m;
#pragma unroll
              for (int v = 0; v < 4; ++v) {
                const int r = rb + M::row(lane, v);
                if (r < m) {
                  T x = cv[u][v];
                  x.x -= accr[v];
                  x.y -= acci[v];
                  Fc[r] = x;
                }
              }
            }
          }
        }
      }
    }
    __syncthreads();
  }
  // Row exchanges -> gather permutation; inverses of the diagonal blocks of
  // L11 (wavefront 0) and U11 (wavefront 1), one block at a time in LDS.
  if (tid == 0) pivots_to_perm(ip, reinterpret_cast<int*>(P), p);
  __syncthreads();
  // Diagonal blocks with leading dimension LDB (32 when every separator of the
  // level fits, so that levels of small separators keep their LDS small), two
  // 64-entry column buffers, then a CR x LDB staging chunk.
  const int LDB = inv_ld(a.max_p);
  T* Db = P;
  for (int j0 = 0; j0 < p; j0 += DIB) {
    const int nbk = min(DIB, p - j0);
    for (int t = tid; t < nbk * nbk; t += NTF) {
      int c = t / nbk, r = t - c * nbk;
      Db[c * LDB + r] = F[(long long)(j0 + c) * m + j0 + r];
    }
    __syncthreads();
    if (wv == 0) invert_lower_unit(Db, LDB, nbk, Db + LDB * LDB, lane);
    if (wv == 1) invert_upper(Db, LDB, nbk, Db + LDB * LDB + 64, lane);
    __syncthreads();
    for (int t = tid; t < nbk * nbk; t += NTF) {
      int c = t / nbk, r = t - c * nbk;
      F[(long long)(j0 + c) * m + j0 + r] = Db[c * LDB + r];
    }
    T* Cb = Db + LDB * LDB + 128;
    // M'_J = -L[j1:m, J] Linv_J, 64 rows at a time.
    const int j1 = j0 + nbk;
    for (int r0 = j1; r0 < m; r0 += CR) {
      const int rows = min(CR, m - r0);
      __syncthreads();
      for (int t = tid; t < rows * nbk; t += NTF) {
        int j = t / rows, rr = t - j * rows;
        Cb[j * CR + rr] = F[(long long)(j0 + j) * m + r0 + rr];
      }
      __syncthreads();
      // [rows x nbk] = -C Linv_J (unit diagonal implicit)
      mma_neg_product<T>(
          rows, nbk, nbk, [&](int r, int k) { return Cb[k * CR + r]; },
          [&](int k, int c) {
            return k == c ? T{(R)1, (R)0} : (k > c ? Db[c * LDB + k] : czero<T>());
          },
          [&](int r, int c, T v) { F[(long long)(j0 + c) * m + r0 + r] = v; }, wv, NTF / 64, lane);
    }
    // N'_J = -U[0:j0, J] Uinv_J, 64 rows at a time.
    for (int r0 = 0; r0 < j0; r0 += CR) {
      const int rows = min(CR, j0 - r0);
      __syncthreads();
      for (int t = tid; t < rows * nbk; t += NTF) {
        int j = t / rows, rr = t - j * rows;
        Cb[j * CR + rr] = F[(long long)(j0 + j) * m + r0 + rr];
      }
      __syncthreads();
      // [rows x nbk] = -C Uinv_J
      mma_neg_product<T>(
          rows, nbk, nbk, [&](int r, int k) { return Cb[k * CR + r]; },
          [&](int k, int c) { return k <= c ? Db[c * LDB + k] : czero<T>(); },
          [&](int r, int c, T v) { F[(long long)(j0 + c) * m + r0 + r] = v; }, wv, NTF / 64, lane);
    }
    // A single-block front also gets V' = -U11^{-1} U12 (64 columns at a time).
    if (p <= DIB) {
      for (int c0 = p; c0 < m; c0 += CR) {
        const int cols = min(CR, m - c0);
        __syncthreads();
        for (int t = tid; t < cols * p; t += NTF) {
          int c = t / p, r = t - c * p;
          Cb[c * LDB + r] = F[(long long)(c0 + c) * m + r];
        }
        __syncthreads();
        // [p x cols] = -Uinv U12
        mma_neg_product<T>(
            p, cols, p, [&](int r, int k) { return k >= r ? Db[k * LDB + r] : czero<T>(); },
            [&](int k, int c) { return Cb[c * LDB + k]; },
            [&](int r, int c, T v) { F[(long long)(c0 + c) * m + r] = v; }, wv, NTF / 64, lane);
      }
    }
    __syncthreads();
  }
  // A separator wider than one block: fold the per-block operators into the
  // full ones, so that every sweep is a single product.  Forward: column block
  // J of [L11^{-1}; -L21 L11^{-1}] collects the phases K > J.  Backward:
  // V' = -U11^{-1} U12 runs through the phases K = last .. 0, then column block
  // J of U11^{-1} collects the phases K < J.  Each pass reads only column
  // blocks that it has not yet rewritten.
  if (p > DIB) {
    const int nJ = (p + DIB - 1) / DIB;
    for (int J = 0; J + 1 < nJ; ++J)
      for (int K = J + 1; K < nJ; ++K)
        fold_step<T, true, NTF>(F, m, K * DIB, min(K * DIB + DIB, p), J * DIB, min(J * DIB + DIB, p), P,
                           tid);
    __syncthreads();
    for (int t = tid; t < p * (m - p); t += NTF) {
      const int c = p + t / p, r = t % p;
      const T x = F[(long long)c * m + r];
      F[(long long)c * m + r] = T{-x.x, -x.y};
    }
    for (int c0 = p; c0 < m; c0 += DIB)
      for (int K = nJ - 1; K >= 0; --K)
        fold_step<T, false, NTF>(F, m, K * DIB, min(K * DIB + DIB, p), c0, min(c0 + DIB, m), P, tid);
    for (int J = nJ - 1; J >= 1; --J)
      for (int K = J - 1; K >= 0; --K)
        fold_step<T, false, NTF>(F, m, K * DIB, min(K * DIB + DIB, p), J * DIB, min(J * DIB + DIB, p), P,
                            tid);
    __syncthreads();
  }
  // Packed sweep operators, a wavefront per column.
  T* Lp = lpk + f.lpk_off;
  for (int k = wv; k < p; k += NTF / 64)
    for (int r = k + 1 + lane; r < m; r += 64) Lp[lpk_col(m, k) + r - k - 1] = F[(long long)k * m + r];
  T* Up = upk + f.upk_off;
  for (int c = wv; c < m; c += NTF / 64) {
    const int rows = c < p ? c + 1 : p;
    for (int r = lane; r < rows; r += 64) Up[upk_col(p, c) + r] = F[(long long)c * m + r];
  }
}

// ---------------------------------------------------------------------------
// Sweeps.  Per front the forward sweep computes
//   y_p = L11^{-1} (P b)_p,   y_q = b_q + M' (P b)_p      (M' = -L21 L11^{-1})
// and the backward sweep
//   x_p = U11^{-1} y_p + V' x_q                          (V' = -U11^{-1} U12),
// so that for p <= DIB each is ONE product with a lower- (forward) or upper-
// (backward) trapezoidal operator.  The operator does not depend on the
// right-hand side: every kernel loads its first operator columns into
// registers before it gathers the vector, so that the chain of dependent loads
// that assembles the right-hand side (descriptor, index maps, values) overlaps
// the bulk of the front's traffic instead of preceding it.
// ---------------------------------------------------------------------------

// sum over k = c0, c0 + step, ... < c1 with k >= cmin of A[ad(k)] x_s[k] for
// NR vectors x_s = x + s xs at once, added to acc[s]: the global loads are
// issued in predicated batches of LB, so that every batch (the last, partial
// one included) costs one memory round trip, and each term is loaded once for
// all right-hand sides.  The column sequence does not depend on the row, so the
// lanes of a wavefront read the same column (contiguous rows) at every step.
template <typename T, int NR, typename Addr>
__device__ inline void gather_dot_nr(const T* __restrict__ A, Addr ad, int c0, int cmin, int c1,
                                     int step, const T* x, int xs, T (&acc)[NR]) {
  constexpr int LB = 8;
  for (int c = c0; c < c1; c += LB * step) {
    T av[LB];
#pragma unroll
    for (int t = 0; t < LB; ++t) {
      const int k = c + t * step;
      av[t] = (k >= cmin && k < c1) ? A[ad(k)] : czero<T>();
    }
#pragma unroll
    for (int t = 0; t < LB; ++t) {
      const int k = c + t * step;
      if (k >= cmin && k < c1)
#pragma unroll
        for (int s = 0; s < NR; ++s) acc[s] = cfma(av[t], x[s * xs + k], acc[s]);
    }
  }
}

// The first KP terms of a strided dot product, A[ad(k0 + G t)] for t < KP and
// kmin <= k0 + G t < kend, held in registers; dot_nr() forms the whole sum for
// NR right-hand sides, taking the terms beyond the first KP from memory (once
// for all of them).
template <typename T, int KP>
struct ColPrefetch {
  T av[KP];
  template <typename Addr>
  __device__ inline void load(const T* __restrict__ A, Addr ad, int k0, int kmin, int kend, int G) {
#pragma unroll
    for (int t = 0; t < KP; ++t) {
      const int k = k0 + G * t;
      av[t] = (k >= kmin && k < kend) ? A[ad(k)] : czero<T>();
    }
  }
  // acc[s] = sum over k = k0, k0 + G, ... < kend with k >= kmin of A[ad(k)] x_s[k]
  template <int NR, typename Addr>
  __device__ inline void dot_nr(const T* __restrict__ A, Addr ad, int k0, int kmin, int kend, int G,
                                const T* x, int xs, T (&acc)[NR]) const {
#pragma unroll
    for (int s = 0; s < NR; ++s) acc[s] = czero<T>();
#pragma unroll
    for (int t = 0; t < KP; ++t) {
      const int k = k0 + G * t;
      if (k >= kmin && k < kend)
#pragma unroll
        for (int s = 0; s < NR; ++s) acc[s] = cfma(av[t], x[s * xs + k], acc[s]);
    }
    const int kt = k0 + G * KP;
    if (kt < kend) gather_dot_nr<T, NR>(A, ad, kt, kmin, kend, G, x, xs, acc);
  }
};

// Forward sweep of one front on one wavefront, for fronts with m <= 64 RPL and
// p <= 64.  Lane rows r = lane + 64 i (i < RPL); with RPL = 1 and m <= 32,
// G = 64 / W lanes share a row (columns k = g, g + G, ...) and a fixed
// butterfly adds their sums.  The NR right-hand sides share the operator
// registers and the index loads.  sh: this wavefront's LDS scratch.
// FUSED (subtree sweeps): the children's update vectors come from the LDS
// slots sl.z, sl.w of the subtree (NR x q_child entries each) and the front's
// own update part goes to its slot sl.y, or to its global front vector when
// sl.y < 0 (the subtree's root); the separator part y_p always goes to the
// global front vector (the backward sweep reads it).
template <typename T, int RPL, int KP, int NR, bool FUSED>
__device__ inline void fwd_front(const LevelArgs& a, const FrontDev& f, const T* __restrict__ lpk,
                                 const int* __restrict__ piv, T* __restrict__ vec, const RhsSet& rs,
                                 T (&sh)[NR][64 * RPL], T* __restrict__ slots, int4 sl) {
  constexpr int MW = 64 * RPL;
  const int lane = threadIdx.x & 63;
  const int m = f.p + f.q, p = f.p, q = f.q;
  const T* L = lpk + f.lpk_off;
  const int W = RPL > 1 ? 64 : (m <= 16 ? 16 : (m <= 32 ? 32 : 64));
  const int G = 64 / W, g = lane / W, rl = lane - g * W;
  ColPrefetch<T, KP> pf[RPL];
#pragma unroll
  for (int i = 0; i < RPL; ++i) {
    const int r = rl + 64 * i;
    pf[i].load(L, LowerAt{m, r}, g, 0, r < m ? min(r, p) : 0, G);
  }
  const int pv = lane < p ? piv[f.piv_off + lane] : lane;
  // b = R^I v on the separator rows plus the children's update vectors (all
  // loaded before any is added).
  long long gidx = -1;
  if (lane < p) {
    const int gx = f.gx0 + lane % f.sw, gy = f.gy0 + lane / f.sw;
    if (gx >= f.ix0 && gx < f.ix1 && gy >= f.iy0 && gy < f.iy1)
      gidx = f.gbase + (long long)gy * f.gnx + gx;
  }
  int d0[RPL], d1[RPL];
#pragma unroll
  for (int i = 0; i < RPL; ++i) {
    const int idx = lane + 64 * i;
    d0[i] = (f.nchild > 0 && idx < f.cq[0]) ? a.cmap[f.ccmap[0] + idx] : -1;
    d1[i] = (f.nchild > 1 && idx < f.cq[1]) ? a.cmap[f.ccmap[1] + idx] : -1;
  }
  T val[NR], c0[NR][RPL], c1[NR][RPL];
#pragma unroll
  for (int s = 0; s < NR; ++s) {
    const T* vs = vec + s * rs.vec_stride;
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      const int idx = lane + 64 * i;
      // predicated on the position, not on the loaded index: the value load
      // does not wait for the child map
      if (FUSED) {
        c0[s][i] = (f.nchild > 0 && idx < f.cq[0]) ? slots[sl.z * NR + s * f.cq[0] + idx] : czero<T>();
        c1[s][i] = (f.nchild > 1 && idx < f.cq[1]) ? slots[sl.w * NR + s * f.cq[1] + idx] : czero<T>();
      } else {
        c0[s][i] = (f.nchild > 0 && idx < f.cq[0]) ? vs[f.cvec[0] + idx] : czero<T>();
        c1[s][i] = (f.nchild > 1 && idx < f.cq[1]) ? vs[f.cvec[1] + idx] : czero<T>();
      }
    }
  }
  // R^I v last: its conversion to T waits for every load issued before it.
#pragma unroll
  for (int s = 0; s < NR; ++s) val[s] = gidx >= 0 ? from_d2<T>(rs.v[s][gidx]) : czero<T>();
#pragma unroll
  for (int s = 0; s < NR; ++s) {
    sh[s][lane] = val[s];
#pragma unroll
    for (int i = 1; i < RPL; ++i) sh[s][lane + 64 * i] = czero<T>();
  }
  wave_sync();
#pragma unroll
  for (int s = 0; s < NR; ++s)
#pragma unroll
    for (int i = 0; i < RPL; ++i)
      if (d0[i] >= 0) sh[s][d0[i]] = cadd(sh[s][d0[i]], c0[s][i]);
  wave_sync();
#pragma unroll
  for (int s = 0; s < NR; ++s)
#pragma unroll
    for (int i = 0; i < RPL; ++i)
      if (d1[i] >= 0) sh[s][d1[i]] = cadd(sh[s][d1[i]], c1[s][i]);
  wave_sync();
  // (P b)_r = b[perm[r]] on the separator rows (p <= 64).
  T pb[NR];
#pragma unroll
  for (int s = 0; s < NR; ++s) pb[s] = sh[s][pv];
  wave_sync();
#pragma unroll
  for (int s = 0; s < NR; ++s) sh[s][lane] = pb[s];
  wave_sync();
#pragma unroll
  for (int i = 0; i < RPL; ++i) {
    const int r = rl + 64 * i;
    const int kend = r < m ? min(r, p) : 0;
    T acc[NR];
    pf[i].template dot_nr<NR>(L, LowerAt{m, r}, g, 0, kend, G, &sh[0][0], MW, acc);
#pragma unroll
    for (int s = 0; s < NR; ++s) {
      if (RPL == 1)
        for (int o = W; o < 64; o <<= 1) acc[s] = cadd(acc[s], shfl_xor_c(acc[s], o));
      if (g == 0 && r < m) {
        const T y = cadd(sh[s][r], acc[s]);
        if (!FUSED || r < p || sl.y < 0) vec[s * rs.vec_stride + f.vec_off + r] = y;
        else slots[sl.y * NR + s * q + (r - p)] = y;
      }
    }
  }
}

// Forward sweep for levels with m <= 64 RPL and p <= 64: four fronts per
// workgroup, one wavefront per front, no workgroup barriers.
template <typename T, int RPL, int KP, int NR>
__global__ __launch_bounds__(NT) void k_fwd_wave(LevelArgs a, const T* __restrict__ lpk,
                                                 const int* __restrict__ piv, T* __restrict__ vec,
                                                 RhsSet rs) {
  __shared__ T sh[4][NR][64 * RPL];
  const int wv = threadIdx.x >> 6;
  const int fi = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + wv);   // uniform per wavefront
  if (fi >= a.nlevel) return;                          // whole wavefront
  const FrontDev f = a.fronts[a.flist ? a.flist[a.first + fi] : a.first + fi];
  if (a.pact && a.pact[f.prob] == 0) return;           // problem converged (whole wavefront)
  fwd_front<T, RPL, KP, NR, false>(a, f, lpk, piv, vec, rs, sh[wv], nullptr, int4{-1, -1, -1, -1});
}

// Backward sweep of one front on one wavefront, for fronts with m <= 128 and
// p <= 64.  Row r < p is shared by G = 64 / W lanes (W >= p), which take
// columns c = r + g, r + g + G, ... of the packed operator [U11^{-1} V'] (ld
// p); a fixed butterfly adds their sums.  FUSED: x_q comes from the front's
// LDS slot sl.y (global front vector when sl.y < 0, the subtree's root) and
// the children's x_q go to their slots sl.z, sl.w instead of their global
// front vectors.
template <typename T, int KP, int NR, bool FUSED>
__device__ inline void bwd_front(const LevelArgs& a, const FrontDev& f, const T* __restrict__ upk,
                                 T* __restrict__ vec, T* __restrict__ u, const RhsSet& rs,
                                 T (&sh)[NR][128], T* __restrict__ slots, int4 sl) {
  const int lane = threadIdx.x & 63;
  const int m = f.p + f.q, p = f.p, q = f.q;
  const T* U = upk + f.upk_off;
  const int W = p <= 4 ? 4 : (p <= 8 ? 8 : (p <= 16 ? 16 : (p <= 32 ? 32 : 64)));
  const int G = 64 / W, g = lane / W, r = lane - g * W;
  ColPrefetch<T, KP> pf;
  pf.load(U, UpperAt{p, r}, g, r, r < p ? m : 0, G);
  const int var = lane < p ? a.vars[f.var_off + lane] : 0;
  // The children's maps (a child's update rows are rows of this front, so
  // q_child <= m <= 128), for the scatter of this front's vector at the end.
  int cm[2][2];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int idx = lane + 64 * i;
      cm[c][i] = (c < f.nchild && idx < f.cq[c]) ? a.cmap[f.ccmap[c] + idx] : -1;
    }
  // [y_p ; x_q]: y_p from the forward sweep, x_q put there by the parent's
  // backward sweep.
  const bool xq_lds = FUSED && sl.y >= 0;
  T y[NR], xq[NR][2];
#pragma unroll
  for (int s = 0; s < NR; ++s) {
    const T* vs = vec + s * rs.vec_stride + f.vec_off;
    y[s] = lane < p ? vs[lane] : czero<T>();
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int idx = lane + 64 * i;
      if (xq_lds) xq[s][i] = idx < q ? slots[sl.y * NR + s * q + idx] : czero<T>();
      else xq[s][i] = idx < q ? vs[p + idx] : czero<T>();
    }
  }
#pragma unroll
  for (int s = 0; s < NR; ++s) {
    if (lane < p) sh[s][lane] = y[s];
#pragma unroll
    for (int i = 0; i < 2; ++i)
      if (lane + 64 * i < q) sh[s][p + lane + 64 * i] = xq[s][i];
  }
  wave_sync();
  const long long uo = a.subs[f.sub].u_off;
  T xp[NR];
  pf.template dot_nr<NR>(U, UpperAt{p, r}, g, r, r < p ? m : 0, G, &sh[0][0], 128, xp);
#pragma unroll
  for (int s = 0; s < NR; ++s)
    for (int o = W; o < 64; o <<= 1) xp[s] = cadd(xp[s], shfl_xor_c(xp[s], o));
  wave_sync();
#pragma unroll
  for (int s = 0; s < NR; ++s)
    if (lane < p) {                        // lane < p <= W: g = 0, r = lane
      sh[s][lane] = xp[s];
      u[s * rs.u_stride + uo + var] = xp[s];
    }
  wave_sync();
  // This front's vector [x_p ; x_q] into the update slots of its children.
#pragma unroll
  for (int s = 0; s < NR; ++s)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int i = 0; i < 2; ++i)
        if (cm[c][i] >= 0) {
          const T x = sh[s][cm[c][i]];
          if (FUSED) slots[(c == 0 ? sl.z : sl.w) * NR + s * f.cq[c] + lane + 64 * i] = x;
          else vec[s * rs.vec_stride + f.cvec[c] + lane + 64 * i] = x;
        }
}

// Backward sweep for levels with m <= 128 and p <= 64: four fronts per
// workgroup, one wavefront per front.
template <typename T, int KP, int NR>
__global__ __launch_bounds__(NT) void k_bwd_wave(LevelArgs a, const T* __restrict__ upk,
                                                 T* __restrict__ vec, T* __restrict__ u, RhsSet rs) {
  __shared__ T sh[4][NR][128];
  const int wv = threadIdx.x >> 6;
  const int fi = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + wv);   // uniform per wavefront
  if (fi >= a.nlevel) return;
  const FrontDev f = a.fronts[a.flist ? a.flist[a.first + fi] : a.first + fi];
  if (a.pact && a.pact[f.prob] == 0) return;           // problem converged (whole wavefront)
  bwd_front<T, KP, NR, false>(a, f, upk, vec, u, rs, sh[wv], nullptr, int4{-1, -1, -1, -1});
}

// ---------------------------------------------------------------------------
// Subtree sweeps: one workgroup (four wavefronts) per group of subtrees of
// the deep levels (a subtree: a front at depth D with all its descendants,
// every level of which the wavefront kernels take).  The fronts are swept level by level
// inside the workgroup (bottom-up forward, top-down backward, a wavefront per
// front, a workgroup barrier between levels), and the update vectors passed
// between them stay in LDS: only the separator parts y_p, the local fields
// and the root's update vector go through global memory.  lev: per subtree,
// K + 1 offsets into fl (relative level j = depth - D); fl: {front, its slot,
// child 0's slot, child 1's slot}, slots in units of q entries (x NR).
// ---------------------------------------------------------------------------
template <typename T, int RPL, int KP, int NR>
__global__ __launch_bounds__(NT) void k_fwd_subtree(LevelArgs a, FuseArgs z, const T* __restrict__ lpk,
                                                    const int* __restrict__ piv, T* __restrict__ vec,
                                                    RhsSet rs) {
  __shared__ T sh[4][NR][64 * RPL];
  extern __shared__ unsigned char smem_raw[];
  T* slots = reinterpret_cast<T*>(smem_raw);
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int* lev = z.lev + (long long)blockIdx.x * (z.K + 1);
  for (int j = z.K - 1; j >= 0; --j) {
    const int e1 = lev[j + 1];
    for (int e = lev[j] + wv; e < e1; e += 4) {
      const int4 sl = z.fl[e];
      const FrontDev f = a.fronts[sl.x];
      // a converged problem's fronts are skipped (a subtree is one problem's)
      if (a.pact && a.pact[f.prob] == 0) continue;
      fwd_front<T, RPL, KP, NR, true>(a, f, lpk, piv, vec, rs, sh[wv], slots, sl);
      wave_sync();
    }
    __syncthreads();
  }
}

template <typename T, int KP, int NR>
__global__ __launch_bounds__(NT) void k_bwd_subtree(LevelArgs a, FuseArgs z, const T* __restrict__ upk,
                                                    T* __restrict__ vec, T* __restrict__ u, RhsSet rs) {
  __shared__ T sh[4][NR][128];
  extern __shared__ unsigned char smem_raw[];
  T* slots = reinterpret_cast<T*>(smem_raw);
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int* lev = z.lev + (long long)blockIdx.x * (z.K + 1);
  for (int j = 0; j < z.K; ++j) {
    const int e1 = lev[j + 1];
    for (int e = lev[j] + wv; e < e1; e += 4) {
      const int4 sl = z.fl[e];
      const FrontDev f = a.fronts[sl.x];
      if (a.pact && a.pact[f.prob] == 0) continue;    // converged problem
      bwd_front<T, KP, NR, true>(a, f, upk, vec, u, rs, sh[wv], slots, sl);
      wave_sync();
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Sweeps, large fronts: one workgroup of NTL threads per front, the single
// trapezoidal product with the first KP operator terms of each thread
// prefetched into registers and shared by the NR right-hand sides.  Rows are
// shared by G = NTL / rows threads (column groups) whose partial sums are
// added in a fixed order through LDS.
// ---------------------------------------------------------------------------
template <typename T, int NTL, int KP, int NR>
__global__ __launch_bounds__(NTL) void k_fwd_large(LevelArgs a, const T* __restrict__ lpk,
                                                   const int* __restrict__ piv, T* __restrict__ vec,
                                                   RhsSet rs) {
  extern __shared__ unsigned char smem_raw[];
  T* scr = reinterpret_cast<T*>(smem_raw);                 // NR x NTL
  T* vl = scr + NR * NTL;                                  // NR x max_m
  T* tmp = vl + NR * a.max_m;                              // NR x max_m
  const int mm = a.max_m;
  const FrontDev f = a.fronts[a.flist ? a.flist[a.first + blockIdx.x] : a.first + blockIdx.x];
  if (a.pact && a.pact[f.prob] == 0) return;           // problem converged (whole workgroup)
  const int m = f.p + f.q, p = f.p;
  const T* L = lpk + f.lpk_off;
  const int tid = threadIdx.x;
  // Rows [r0, r1) of the product: part blockIdx.y of gridDim.y (every part
  // stages the whole right-hand side).
  const int chunk = (m + gridDim.y - 1) / gridDim.y;
  const int r0 = blockIdx.y * chunk, r1 = min(m, r0 + chunk), R = r1 - r0;
  if (R <= 0) return;                                      // whole workgroup
  int G = 1, g = 0, rr = r0 + tid;
  if (R < NTL) {
    G = NTL / R;
    g = tid / R;
    rr = r0 + tid - g * R;
  }
  const bool act = g < G && rr < r1;
  ColPrefetch<T, KP> pf;
  pf.load(L, LowerAt{m, rr}, g, 0, act ? min(rr, p) : 0, G);
  const int* perm = piv + f.piv_off;
  auto global_row = [&](int i) -> long long {
    const int gx = f.gx0 + i % f.sw, gy = f.gy0 + i / f.sw;
    return (gx >= f.ix0 && gx < f.ix1 && gy >= f.iy0 && gy < f.iy1)
               ? f.gbase + (long long)gy * f.gnx + gx
               : -1;
  };
  if (m <= 2 * NTL) {
    // Every global load of the right-hand side first (two rows per thread),
    // so that the chains (index -> value) of R^I v, of both children's update
    // vectors and of the pivots overlap; then the extend-add in LDS.
    long long gidx[2];
    int d0[2], d1[2], pv[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int i = tid + u * NTL;
      gidx[u] = i < p ? global_row(i) : -1;
      d0[u] = (f.nchild > 0 && i < f.cq[0]) ? a.cmap[f.ccmap[0] + i] : -1;
      d1[u] = (f.nchild > 1 && i < f.cq[1]) ? a.cmap[f.ccmap[1] + i] : -1;
      pv[u] = i < p ? perm[i] : -1;
    }
    T bv[2][NR], c0[2][NR], c1[2][NR];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int i = tid + u * NTL;
#pragma unroll
      for (int s = 0; s < NR; ++s) {
        const T* vs = vec + s * rs.vec_stride;
        // predicated on the position, not on the loaded index (no chain)
        c0[u][s] = (f.nchild > 0 && i < f.cq[0]) ? vs[f.cvec[0] + i] : czero<T>();
        c1[u][s] = (f.nchild > 1 && i < f.cq[1]) ? vs[f.cvec[1] + i] : czero<T>();
      }
    }
    // R^I v last: its conversion to T waits for every load issued before it.
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int s = 0; s < NR; ++s)
        bv[u][s] = gidx[u] >= 0 ? from_d2<T>(rs.v[s][gidx[u]]) : czero<T>();
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int i = tid + u * NTL;
      if (i < m)
#pragma unroll
        for (int s = 0; s < NR; ++s) vl[s * mm + i] = bv[u][s];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 2; ++u)
      if (d0[u] >= 0)
#pragma unroll
        for (int s = 0; s < NR; ++s) vl[s * mm + d0[u]] = cadd(vl[s * mm + d0[u]], c0[u][s]);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 2; ++u)
      if (d1[u] >= 0)
#pragma unroll
        for (int s = 0; s < NR; ++s) vl[s * mm + d1[u]] = cadd(vl[s * mm + d1[u]], c1[u][s]);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 2; ++u)
      if (pv[u] >= 0)
#pragma unroll
        for (int s = 0; s < NR; ++s) tmp[s * mm + tid + u * NTL] = vl[s * mm + pv[u]];
  } else {
    for (int i = tid; i < m; i += NTL) {
      const long long gi = i < p ? global_row(i) : -1;
#pragma unroll
      for (int s = 0; s < NR; ++s) vl[s * mm + i] = gi >= 0 ? from_d2<T>(rs.v[s][gi]) : czero<T>();
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      if (f.nchild > c) {
        const int* cm = a.cmap + f.ccmap[c];
        for (int i = tid; i < f.cq[c]; i += NTL) {
          const int d = cm[i];
#pragma unroll
          for (int s = 0; s < NR; ++s)
            vl[s * mm + d] = cadd(vl[s * mm + d], vec[s * rs.vec_stride + f.cvec[c] + i]);
        }
        __syncthreads();
      }
    }
    for (int i = tid; i < p; i += NTL) {
      const int src = perm[i];
#pragma unroll
      for (int s = 0; s < NR; ++s) tmp[s * mm + i] = vl[s * mm + src];
    }
  }
  __syncthreads();
  for (int i = tid; i < p; i += NTL)
#pragma unroll
    for (int s = 0; s < NR; ++s) vl[s * mm + i] = tmp[s * mm + i];
  __syncthreads();
  T acc[NR];
  pf.template dot_nr<NR>(L, LowerAt{m, rr}, g, 0, act ? min(rr, p) : 0, G, vl, mm, acc);
  if (G == 1) {
    if (act)
#pragma unroll
      for (int s = 0; s < NR; ++s) vec[s * rs.vec_stride + f.vec_off + rr] = cadd(vl[s * mm + rr], acc[s]);
    for (int r = rr + NTL; r < r1; r += NTL) {
      T ext[NR];
#pragma unroll
      for (int s = 0; s < NR; ++s) ext[s] = czero<T>();
      gather_dot_nr<T, NR>(L, LowerAt{m, r}, 0, 0, min(r, p), 1, vl, mm, ext);
#pragma unroll
      for (int s = 0; s < NR; ++s) vec[s * rs.vec_stride + f.vec_off + r] = cadd(vl[s * mm + r], ext[s]);
    }
  } else {
#pragma unroll
    for (int s = 0; s < NR; ++s) scr[s * NTL + tid] = acc[s];
    __syncthreads();
    if (tid < R) {
#pragma unroll
      for (int s = 0; s < NR; ++s) {
        T sum = czero<T>();
        for (int gg = 0; gg < G; ++gg) sum = cadd(sum, scr[s * NTL + gg * R + tid]);
        vec[s * rs.vec_stride + f.vec_off + r0 + tid] = cadd(vl[s * mm + r0 + tid], sum);
      }
    }
  }
}

template <typename T, int NTL, int KP, int NR>
__global__ __launch_bounds__(NTL) void k_bwd_large(LevelArgs a, const T* __restrict__ upk,
                                                   T* __restrict__ vec, T* __restrict__ u, RhsSet rs) {
  extern __shared__ unsigned char smem_raw[];
  T* scr = reinterpret_cast<T*>(smem_raw);                 // NR x NTL
  T* vl = scr + NR * NTL;                                  // NR x max_m
  const int mm = a.max_m;
  const FrontDev f = a.fronts[a.flist ? a.flist[a.first + blockIdx.x] : a.first + blockIdx.x];
  if (a.pact && a.pact[f.prob] == 0) return;           // problem converged (whole workgroup)
  const int m = f.p + f.q, p = f.p;
  const T* U = upk + f.upk_off;                            // packed [U11^{-1} V']
  const int tid = threadIdx.x;
  // Rows [r0, r1) of x_p: part blockIdx.y of gridDim.y.  Every part stages the
  // whole [y_p ; x_q]; part 0 also passes x_q on to the children.  A part never
  // writes this front's own vector (the host keeps R <= NTL when there are
  // several parts), which the other parts read.
  const int sp = blockIdx.y;
  const int chunk = (p + gridDim.y - 1) / gridDim.y;
  const int r0 = sp * chunk, r1 = min(p, r0 + chunk), R = r1 - r0;
  if (R <= 0) return;                                      // whole workgroup (never part 0)
  int G = 1, g = 0, rr = r0 + tid;
  if (R < NTL) {
    G = NTL / R;
    g = tid / R;
    rr = r0 + tid - g * R;
  }
  const bool act = g < G && rr < r1;
  ColPrefetch<T, KP> pf;
  pf.load(U, UpperAt{p, rr}, g, rr, act ? m : 0, G);
  const int* vars = a.vars + f.var_off;
  // the row this thread stores: rr (one column group) or r0 + tid (summed groups)
  const int row = G == 1 ? rr : r0 + tid;
  const bool has_row = G == 1 ? act : tid < R;
  const int var = has_row ? vars[row] : 0;
  // The children's maps (issued early; two entries per thread, the rest later).
  int cm[2][2];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int idx = tid + NTL * i;
      cm[c][i] = (c < f.nchild && idx < f.cq[c]) ? a.cmap[f.ccmap[c] + idx] : -1;
    }
  // [y_p ; x_q]: this front's own vector (x_q put there by the parent).
  for (int i = tid; i < m; i += NTL)
#pragma unroll
    for (int s = 0; s < NR; ++s) vl[s * mm + i] = vec[s * rs.vec_stride + f.vec_off + i];
  __syncthreads();
  const long long uo = a.subs[f.sub].u_off;
  T acc[NR];
  pf.template dot_nr<NR>(U, UpperAt{p, rr}, g, rr, act ? m : 0, G, vl, mm, acc);
  if (G == 1) {
    // rows beyond NTL (p > NTL): written to the front vector now, read back below
    for (int r = rr + NTL; r < r1; r += NTL) {
      T x[NR];
#pragma unroll
      for (int s = 0; s < NR; ++s) x[s] = czero<T>();
      gather_dot_nr<T, NR>(U, UpperAt{p, r}, 0, r, m, 1, vl, mm, x);
      const int vr = vars[r];
#pragma unroll
      for (int s = 0; s < NR; ++s) {
        vec[s * rs.vec_stride + f.vec_off + r] = x[s];
        u[s * rs.u_stride + uo + vr] = x[s];
      }
    }
  } else {
#pragma unroll
    for (int s = 0; s < NR; ++s) scr[s * NTL + tid] = acc[s];
    __syncthreads();
    if (tid < R) {
#pragma unroll
      for (int s = 0; s < NR; ++s) {
        T sum = czero<T>();
        for (int gg = 0; gg < G; ++gg) sum = cadd(sum, scr[s * NTL + gg * R + tid]);
        acc[s] = sum;
      }
    }
  }
  __syncthreads();                        // every read of y_p by the products is done
  if (has_row)
#pragma unroll
    for (int s = 0; s < NR; ++s) {
      vl[s * mm + row] = acc[s];
      u[s * rs.u_stride + uo + var] = acc[s];
    }
  for (int r = rr + NTL; G == 1 && r < r1; r += NTL)
#pragma unroll
    for (int s = 0; s < NR; ++s) vl[s * mm + r] = vec[s * rs.vec_stride + f.vec_off + r];
  __syncthreads();
  // This front's vector [x_p ; x_q] into the update slots of its children:
  // the rows of x_p this part computed, and x_q from part 0.
  auto mine = [&](int d) { return d >= p ? sp == 0 : (d >= r0 && d < r1); };
#pragma unroll
  for (int c = 0; c < 2; ++c) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
      if (cm[c][i] >= 0 && mine(cm[c][i]))
#pragma unroll
        for (int s = 0; s < NR; ++s)
          vec[s * rs.vec_stride + f.cvec[c] + tid + NTL * i] = vl[s * mm + cm[c][i]];
    if (c < f.nchild)
      for (int idx = tid + 2 * NTL; idx < f.cq[c]; idx += NTL) {
        const int d = a.cmap[f.ccmap[c] + idx];
        if (mine(d))
#pragma unroll
          for (int s = 0; s < NR; ++s) vec[s * rs.vec_stride + f.cvec[c] + idx] = vl[s * mm + d];
      }
  }
}

// z_s = sum_k P_k u_k for each right-hand side s: each global node adds the
// local fields of the (at most four) subdomains whose Omega_k covers it, in a
// fixed order.
template <typename T, int NR>
__global__ __launch_bounds__(256) void k_scatter(const T* __restrict__ u, const SubDev* __restrict__ subs,
                                                 const int4* __restrict__ cover_x,
                                                 const int4* __restrict__ cover_y,
                                                 const ScatDev* __restrict__ probs,
                                                 const int* __restrict__ pact, RhsSet rs) {
  const ScatDev P = probs[blockIdx.z];
  if (pact && pact[blockIdx.z] == 0) return;
  const int nx = P.nx, ny = P.ny, px = P.px;
  int i = blockIdx.x * 64 + threadIdx.x;
  int j = blockIdx.y * 4 + threadIdx.y;
  if (i >= nx || j >= ny) return;
  subs += P.sub0;
  int4 cx = cover_x[P.cx_off + i], cy = cover_y[P.cy_off + j];
  double2 acc[NR];
#pragma unroll
  for (int s = 0; s < NR; ++s) acc[s] = make_double2(0.0, 0.0);
  int kys[2] = {cy.x, cy.z}, uys[2] = {cy.y, cy.w};
  int kxs[2] = {cx.x, cx.z}, txs[2] = {cx.y, cx.w};
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    if (kys[b] < 0) continue;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      if (kxs[c] < 0) continue;
      const SubDev& s = subs[kys[b] * px + kxs[c]];
      const long long o = s.u_off + (long long)uys[b] * s.nxl + txs[c];
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        double2 val = to_d2(u[r * rs.u_stride + o]);
        acc[r].x += val.x;
        acc[r].y += val.y;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) rs.z[r][P.gbase + (long long)j * nx + i] = acc[r];
}

// ---------------------------------------------------------------------------
// Staged (multiplicative) order of the round.  A stage solves its subdomains
// with the residual the earlier stages left: r = v - A z on their own boxes I_k
// (disjoint), the usual sweeps on their fronts only, then z += sum of their
// full local fields.  Blocks of 64 x 4 nodes, blockIdx.z = the stage member.
// ---------------------------------------------------------------------------
template <int NR>
__global__ __launch_bounds__(256) void k_stage_residual(const double2* __restrict__ keps,
                                                        const double2* __restrict__ gc,
                                                        const SubDev* __restrict__ subs,
                                                        const ScatDev* __restrict__ probs,
                                                        const int* __restrict__ slist, int sfirst,
                                                        const int* __restrict__ pact, RhsSet rs,
                                                        double2* __restrict__ rbuf,
                                                        long long rstride) {
  const SubDev S = subs[slist[sfirst + blockIdx.z]];
  if (pact && pact[S.prob] == 0) return;
  const int gx = S.ix0 + blockIdx.x * 64 + threadIdx.x;
  const int gy = S.iy0 + blockIdx.y * 4 + threadIdx.y;
  if (gx >= S.ix1 || gy >= S.iy1) return;
  const ScatDev P = probs[S.prob];
  const int nx = P.nx, ny = P.ny;
  const double2* cxw = gc + P.gc_off;
  const double2* cxe = cxw + nx;
  const double2* cyw = cxe + nx;
  const double2* cye = cyw + ny;
  const long long n = P.gbase + (long long)gy * nx + gx;
  const double2 aw = cxw[gx], ae = cxe[gx], as = cyw[gy], an = cye[gy];
  const double2 ke = keps[n];
  const double2 dg = make_double2(ke.x - ((aw.x + ae.x) + (as.x + an.x)),
                                  ke.y - ((aw.y + ae.y) + (as.y + an.y)));
#pragma unroll
  for (int s = 0; s < NR; ++s) {
    const double2* z = rs.z[s];
    double2 acc = cmul(dg, z[n]);
    if (gx > 0) acc = cfma(aw, z[n - 1], acc);
    if (gx < nx - 1) acc = cfma(ae, z[n + 1], acc);
    if (gy > 0) acc = cfma(as, z[n - nx], acc);
    if (gy < ny - 1) acc = cfma(an, z[n + nx], acc);
    rbuf[s * rstride + n] = csub(rs.v[s][n], acc);
  }
}

template <typename T, int NR>
__global__ __launch_bounds__(256) void k_stage_scatter(const T* __restrict__ u,
                                                       const SubDev* __restrict__ subs,
                                                       const ScatDev* __restrict__ probs,
                                                       const int4* __restrict__ cover_x,
                                                       const int4* __restrict__ cover_y,
                                                       const int* __restrict__ slist, int sfirst,
                                                       const int* __restrict__ inst,
                                                       const int* __restrict__ pact, RhsSet rs) {
  const int k = slist[sfirst + blockIdx.z];
  const SubDev S = subs[k];
  if (pact && pact[S.prob] == 0) return;
  const int gx = S.ox0 + blockIdx.x * 64 + threadIdx.x;
  const int gy = S.oy0 + blockIdx.y * 4 + threadIdx.y;
  if (gx >= S.ox0 + S.nxl || gy >= S.oy0 + S.nyl) return;
  const ScatDev P = probs[S.prob];
  const int4 cx = cover_x[P.cx_off + gx], cy = cover_y[P.cy_off + gy];
  const int kys[2] = {cy.x, cy.z}, uys[2] = {cy.y, cy.w};
  const int kxs[2] = {cx.x, cx.z}, txs[2] = {cx.y, cx.w};
  // The stage members covering this node; the lowest one adds them all.
  int mem[4], loc[4], cnt = 0, low = 1 << 30;
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      if (kys[b] < 0 || kxs[c] < 0) continue;
      const int kk = P.sub0 + kys[b] * P.px + kxs[c];
      if (inst[kk] == 0) continue;
      const SubDev& Q = subs[kk];
      mem[cnt] = kk;
      loc[cnt] = uys[b] * Q.nxl + txs[c];
      low = kk < low ? kk : low;
      ++cnt;
    }
  if (low != k) return;
  const long long n = P.gbase + (long long)gy * P.nx + gx;
#pragma unroll
  for (int s = 0; s < NR; ++s) {
    double2 acc = rs.z[s][n];
    for (int i = 0; i < cnt; ++i) {
      const double2 v = to_d2(u[s * rs.u_stride + subs[mem[i]].u_off + loc[i]]);
      acc.x += v.x;
      acc.y += v.y;
    }
    rs.z[s][n] = acc;
  }
}

// The first stage's sum over the whole grid (blockIdx.z = problem): z_s =
// the sum of the local fields of the stage's members covering the node, in
// the fixed order of k_stage_scatter (0 where none covers it), so that z needs
// no zero fill before the application.
template <typename T, int NR>
__global__ __launch_bounds__(256) void k_stage_scatter_first(const T* __restrict__ u,
                                                             const SubDev* __restrict__ subs,
                                                             const int4* __restrict__ cover_x,
                                                             const int4* __restrict__ cover_y,
                                                             const ScatDev* __restrict__ probs,
                                                             const int* __restrict__ inst,
                                                             const int* __restrict__ pact, RhsSet rs) {
  const ScatDev P = probs[blockIdx.z];
  const int gx = blockIdx.x * 64 + threadIdx.x;
  const int gy = blockIdx.y * 4 + threadIdx.y;
  if (gx >= P.nx || gy >= P.ny) return;
  const int4 cx = cover_x[P.cx_off + gx], cy = cover_y[P.cy_off + gy];
  const int kys[2] = {cy.x, cy.z}, uys[2] = {cy.y, cy.w};
  const int kxs[2] = {cx.x, cx.z}, txs[2] = {cx.y, cx.w};
  double2 acc[NR];
#pragma unroll
  for (int s = 0; s < NR; ++s) acc[s] = make_double2(0.0, 0.0);
  const bool active = !pact || pact[blockIdx.z] != 0;   // a converged problem's z stays 0
#pragma unroll
  for (int b = 0; b < 2 && active; ++b)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      if (kys[b] < 0 || kxs[c] < 0) continue;
      const int kk = P.sub0 + kys[b] * P.px + kxs[c];
      if (inst[kk] == 0) continue;
      const SubDev& Q = subs[kk];
      const long long o = Q.u_off + (long long)uys[b] * Q.nxl + txs[c];
#pragma unroll
      for (int s = 0; s < NR; ++s) {
        const double2 v = to_d2(u[s * rs.u_stride + o]);
        acc[s].x += v.x;
        acc[s].y += v.y;
      }
    }
  const long long n = P.gbase + (long long)gy * P.nx + gx;
#pragma unroll
  for (int s = 0; s < NR; ++s) rs.z[s][n] = acc[s];
}

__global__ __launch_bounds__(256) void k_zero(double2* __restrict__ p, long long n) {
  for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < n; t += (long long)gridDim.x * 256)
    p[t] = make_double2(0.0, 0.0);
}

// The quantity of Eq. (20): per subdomain (block), the 2-norm of its local
// field on Omega_k outside I_k (the overlapping region), then (one block) the
// sum of those norms over the subdomains in index order.
template <typename T>
__global__ __launch_bounds__(256) void k_overlap_norm(const T* __restrict__ u,
                                                      const SubDev* __restrict__ subs,
                                                      double* __restrict__ per_sub) {
  __shared__ double red[4];
  const SubDev S = subs[blockIdx.x];
  const int n = S.nxl * S.nyl;
  double a = 0.0;
  for (int t = threadIdx.x; t < n; t += 256) {
    const int gx = S.ox0 + t % S.nxl, gy = S.oy0 + t / S.nxl;
    if (gx >= S.ix0 && gx < S.ix1 && gy >= S.iy0 && gy < S.iy1) continue;
    const double2 v = to_d2(u[S.u_off + t]);
    a += v.x * v.x + v.y * v.y;
  }
  a = wave_sum(a);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) per_sub[blockIdx.x] = sqrt((red[0] + red[1]) + (red[2] + red[3]));
}

__global__ __launch_bounds__(64) void k_sum_ordered(const double* __restrict__ a, int n,
                                                    double* __restrict__ out) {
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += a[i];
    out[0] = s;
  }
}

int g_max_lds = 0;
int max_lds() {
  if (g_max_lds == 0) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
        v > 0)
      g_max_lds = v;
    else
      g_max_lds = 163840;          // gfx950: 160 KiB of LDS per workgroup (no device: host checks)
  }
  return g_max_lds;
}

// LDS bytes of the panel kernel with NB-column panels on a level.
size_t panel_lds(const LevelArgs& a, size_t elem, int nb) {
  const size_t ld = inv_ld(a.max_p);
  return std::max((size_t)a.max_m * nb, ld * ld + 128 + (size_t)CR * ld) * elem;
}
// Static LDS of the panel kernel besides the dynamic panel (staged U chunk,
// pivot and reduction arrays), bounded.
size_t panel_static_lds(size_t elem) { return (size_t)UC * 33 * elem + 512; }

template <typename T, int NB, int NTF = NT>
void large_launch(hipStream_t st, const LevelArgs& a, T* fac, T* lpk, T* upk, int* piv, int* flag,
                  double tau) {
  const size_t lds = panel_lds(a, sizeof(T), NB);
  STF_LAUNCH((k_factor_large<T, NB, NTF>), dim3(a.nlevel), dim3(NTF), lds, st, a, fac, lpk,
                     upk, piv, flag, tau);
}

}  // namespace

int g_num_cus = 0;
int num_cus() {
  if (g_num_cus == 0) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        v > 0)
      g_num_cus = v;
    else
      g_num_cus = 256;
  }
  return g_num_cus;
}

int small_factor_limit(size_t elem) {
  // Largest front order whose m x m block (plus two 64-entry buffers) fits
  // 40 KiB of LDS, so that several one-wavefront workgroups share a CU.
  int lim = 1;
  while ((size_t)((lim + 1) * (lim + 1) + 128) * elem <= 40960) ++lim;
  return std::min(lim, 64);
}

// The built-in choice for a level.
FactorShape factor_default(const LevelArgs& a, size_t elem) {
  if (a.max_m <= small_factor_limit(elem)) return FactorShape{1, 0, 64};
  // Panel width: as wide as the LDS allows for the largest front of the level
  // (the staged U chunk and small arrays take the rest).
  const size_t budget = (size_t)max_lds() - panel_static_lds(elem);
  const size_t per_col = (size_t)a.max_m * elem;
  // Fronts of order <= 256: panels as wide as the separator where that fits,
  // so that the Schur complement is updated in fewer passes, except for
  // complex64 fronts of order <= 128, whose levels hold thousands of fronts
  // and keep 8-column panels (fewer registers, more workgroups per CU).
  int nb_max = elem == 16 ? 16 : 32;
  int one = 1;
  while (one < a.max_p) one *= 2;
  if (a.max_m <= 128 && elem == 8) nb_max = 8;
  else if (a.max_m <= 256) nb_max = std::min(nb_max, one);
  int nb = 1;
  while (nb * 2 <= nb_max && per_col * nb * 2 <= budget) nb *= 2;
  if (per_col * nb > budget) throw Error(STF_EINVAL, "front too large for the LDS panel");
  // Levels with at most one front per CU: four times the threads per front
  // (the serial chain of a front is the level's time), with 16-column panels
  // (8 in FP64) so that a thread fits in 128 registers.
  const int nb1k = elem == 8 ? 16 : 8;
  if (a.nlevel <= 256 && nb >= nb1k) return FactorShape{2, nb1k, 1024};
  return FactorShape{2, nb, NT};
}

bool factor_shape_ok(const LevelArgs& a, size_t elem, const FactorShape& s) {
  if (s.kind == 0) return true;
  if (s.kind == 1) return s.ntf == 64 && a.max_m <= small_factor_limit(elem);
  if (s.kind != 2) return false;
  const int nb1k = elem == 8 ? 16 : 8;
  const bool inst = (s.ntf == NT && (s.nb == 1 || s.nb == 2 || s.nb == 4 || s.nb == 8 || s.nb == 16 ||
                                     s.nb == 32)) ||
                    (s.ntf == 1024 && s.nb == nb1k);
  if (!inst) return false;
  if (panel_lds(a, elem, s.nb) + panel_static_lds(elem) > (size_t)max_lds()) return false;
  return true;
}

std::vector<FactorShape> factor_candidates(const LevelArgs& a, size_t elem) {
  std::vector<FactorShape> out;
  const FactorShape d = factor_default(a, elem);
  out.push_back(d);
  auto add = [&](FactorShape s) {
    if (!factor_shape_ok(a, elem, s)) return;
    for (const FactorShape& o : out)
      if (o.kind == s.kind && o.nb == s.nb && o.ntf == s.ntf) return;
    out.push_back(s);
  };
  if (a.max_m <= small_factor_limit(elem)) {
    // the LDS kernel, or the panel kernel with narrow panels
    add(FactorShape{2, 4, NT});
    add(FactorShape{2, 8, NT});
    return out;
  }
  const int nb1k = elem == 8 ? 16 : 8;
  for (int nb : {8, 16, 32}) {
    if (elem == 16 && nb > 16) continue;
    add(FactorShape{2, nb, NT});
  }
  if (a.nlevel <= 4 * num_cus()) add(FactorShape{2, nb1k, 1024});
  return out;
}

template <typename T>
void launch_front_factor(hipStream_t st, const LevelArgs& a, T* fac, T* lpk, T* upk, int* piv, int* flag,
                         double tau, FactorShape sh) {
  if (sh.kind == 0) sh = factor_default(a, sizeof(T));
  if (!factor_shape_ok(a, sizeof(T), sh)) throw Error(STF_EINVAL, "factorisation launch shape not valid for the level");
  if (sh.kind == 1) {
    size_t lds = ((size_t)a.max_m * a.max_m + 128) * sizeof(T);
    STF_LAUNCH(k_factor_small<T>, dim3(a.nlevel), dim3(64), lds, st, a, fac, lpk, upk, piv, flag,
                       tau);
    return;
  }
  if (sh.ntf == 1024) {
    constexpr int NB1K = sizeof(T) == 8 ? 16 : 8;
    large_launch<T, NB1K, 1024>(st, a, fac, lpk, upk, piv, flag, tau);
    return;
  }
  switch (sh.nb) {
    case 32: large_launch<T, 32>(st, a, fac, lpk, upk, piv, flag, tau); break;
    case 16: large_launch<T, 16>(st, a, fac, lpk, upk, piv, flag, tau); break;
    case 8: large_launch<T, 8>(st, a, fac, lpk, upk, piv, flag, tau); break;
    case 4: large_launch<T, 4>(st, a, fac, lpk, upk, piv, flag, tau); break;
    case 2: large_launch<T, 2>(st, a, fac, lpk, upk, piv, flag, tau); break;
    default: large_launch<T, 1>(st, a, fac, lpk, upk, piv, flag, tau); break;
  }
}

// Smallest prefetch depth in {8, 16, 32} that covers `need` columns, capped
// at `cap` (the rest of a row is read by the dot product's tail batches).
inline int prefetch_depth(int need, int cap) {
  int kp = 8;
  while (kp < need && kp < cap) kp *= 2;
  return kp;
}

// Workgroup size for the large-front sweeps: the largest of 256, 512, 1024
// threads with which the level's nwg workgroups all fit in one round at
// sixteen wavefronts per CU (the latency of one front is the level's time, so a
// second round costs more than narrower workgroups do); at least 256.
inline int large_threads(int nwg) {
  const long long budget = 16LL * num_cus();             // resident wavefronts
  int ntl = 256;
  while (ntl < 1024 && (long long)nwg * (2 * ntl / 64) <= budget) ntl *= 2;
  return ntl;
}

// Workgroups per front for the large-front sweeps: a level of fewer fronts
// than CUs splits each front's rows over up to eight parts, until there is a
// workgroup per CU (sixteen wavefronts each), keeping at least 32 rows per
// part; a level that already fills the chip gains nothing from parts, which
// each stage the whole right-hand side.  Several parts only when each takes at
// most 256 rows (<= the workgroup's threads): a part then never writes its
// front's own vector, which the other parts read.
inline int sweep_parts(int nfronts, int rows) {
  int parts = 1;
  while (parts < 8 && (long long)nfronts * parts < num_cus() && rows / (2 * parts) >= 32)
    parts *= 2;
  if (parts > 1 && (rows + parts - 1) / parts > 256) parts = 1;
  return parts;
}

// Instantiation over the number of right-hand sides swept together.
#define STF_NR_DISPATCH(nr, CALL) \
  switch (nr) {                   \
    case 1: CALL(1); break;       \
    case 2: CALL(2); break;       \
    case 3: CALL(3); break;       \
    default: CALL(4); break;      \
  }

template <typename T, int RPL, int KP>
void fwd_wave_launch(hipStream_t st, const LevelArgs& a, const T* fac, const int* piv, T* vec,
                     const RhsSet& r) {
#define STF_CALL(NR) \
  STF_LAUNCH((k_fwd_wave<T, RPL, KP, NR>), dim3((a.nlevel + 3) / 4), dim3(NT), 0, st, a, fac, piv, vec, r)
  STF_NR_DISPATCH(r.nr, STF_CALL)
#undef STF_CALL
}

template <typename T, int KP>
void bwd_wave_launch(hipStream_t st, const LevelArgs& a, const T* upk, T* vec, T* u,
                     const RhsSet& r) {
#define STF_CALL(NR) \
  STF_LAUNCH((k_bwd_wave<T, KP, NR>), dim3((a.nlevel + 3) / 4), dim3(NT), 0, st, a, upk, vec, u, r)
  STF_NR_DISPATCH(r.nr, STF_CALL)
#undef STF_CALL
}

template <typename T, int NTL, int KP>
void fwd_large_nr(hipStream_t st, const LevelArgs& a, int parts, const T* fac, const int* piv,
                  T* vec, const RhsSet& r) {
  const size_t lds = ((size_t)r.nr * NTL + 2 * (size_t)r.nr * a.max_m) * sizeof(T);
#define STF_CALL(NR)                                                                         \
  STF_LAUNCH((k_fwd_large<T, NTL, KP, NR>), dim3(a.nlevel, parts), dim3(NTL), lds, st, a, \
                     fac, piv, vec, r)
  STF_NR_DISPATCH(r.nr, STF_CALL)
#undef STF_CALL
}

template <typename T, int NTL, int KP>
void bwd_large_nr(hipStream_t st, const LevelArgs& a, int parts, const T* upk, T* vec, T* u,
                  const RhsSet& r) {
  const size_t lds = ((size_t)r.nr * NTL + (size_t)r.nr * a.max_m) * sizeof(T);
#define STF_CALL(NR)                                                                         \
  STF_LAUNCH((k_bwd_large<T, NTL, KP, NR>), dim3(a.nlevel, parts), dim3(NTL), lds, st, a, \
                     upk, vec, u, r)
  STF_NR_DISPATCH(r.nr, STF_CALL)
#undef STF_CALL
}

template <typename T, int NTL>
void fwd_large_launch(hipStream_t st, const LevelArgs& a, int parts, int kp, const T* fac,
                      const int* piv, T* vec, const RhsSet& r) {
  if (kp <= 16)
    fwd_large_nr<T, NTL, 16>(st, a, parts, fac, piv, vec, r);
  else
    fwd_large_nr<T, NTL, (sizeof(T) == 8 ? 32 : 16)>(st, a, parts, fac, piv, vec, r);
}

template <typename T, int NTL>
void bwd_large_launch(hipStream_t st, const LevelArgs& a, int parts, int kp, const T* upk,
                      T* vec, T* u, const RhsSet& r) {
  if (kp <= 16)
    bwd_large_nr<T, NTL, 16>(st, a, parts, upk, vec, u, r);
  else
    bwd_large_nr<T, NTL, (sizeof(T) == 8 ? 32 : 16)>(st, a, parts, upk, vec, u, r);
}

void check_rhs(const RhsSet& r) {
  if (r.nr < 1 || r.nr > MAX_RHS) throw Error(STF_EINVAL, "1 to 4 right-hand sides per sweep");
}

// Levels the one-wavefront sweep kernels take: m <= 128 (two rows per lane,
// or a 128-entry vector per wavefront backwards) and p <= 64 (a pivot or
// separator row per lane).
bool wave_level(const LevelArgs& a) { return a.max_m <= 128 && a.max_p <= 64; }

// Instantiated prefetch depths: wavefront kernels 8, 16, 32 (complex64) or
// 8, 16 (complex128), halved for two rows per lane; workgroup kernels 16, 32
// (complex64) or 16.
int wave_kp_max(size_t elem, int rpl) { return (elem == 8 ? 32 : 16) / rpl; }
int large_kp_max(size_t elem) { return elem == 8 ? 32 : 16; }

size_t sweep_lds(const LevelArgs& a, bool fwd, size_t elem, int nr, int ntl) {
  return ((size_t)nr * ntl + (fwd ? 2 : 1) * (size_t)nr * a.max_m) * elem;
}

SweepShape sweep_default(const LevelArgs& a, bool fwd, size_t elem) {
  const int cap = elem == 8 ? 32 : 16;           // registers per lane for the prefetch
  if (wave_level(a)) {
    // Wavefront kernels: at most 16 prefetched terms per lane (about 60
    // registers), so that eight wavefronts per SIMD hide the gather latency.
    if (fwd) {
      // A lane row takes at most min(r, p) <= max_p columns.
      const int rpl = a.max_m <= 64 ? 1 : 2;
      return SweepShape{1, prefetch_depth(a.max_p, 16 / rpl), 64, 1};
    }
    // Row groups: W >= max_p lanes, so G >= 64 / W groups share a row's columns.
    int w = 4;
    while (w < a.max_p) w *= 2;
    const int g = 64 / w;
    return SweepShape{1, prefetch_depth((a.max_m + g - 1) / g, 16), 64, 1};
  }
  if (fwd) {
    // The rows of each front in `parts` workgroups; a row takes at most p columns.
    const int parts = sweep_parts(a.nlevel, a.max_m);
    const int ntl = large_threads(a.nlevel * parts);
    const int rows = (a.max_m + parts - 1) / parts;
    const int g = std::max(1, ntl / rows);
    // A level of more workgroups than one round at four wavefronts per SIMD holds
    // sixteen terms per lane (about 70 registers, seven wavefronts per SIMD).
    const bool many = (long long)a.nlevel * parts * (ntl / 64) > 16LL * num_cus();
    return SweepShape{2, std::max(16, prefetch_depth((a.max_p + g - 1) / g, many ? 16 : cap)), ntl, parts};
  }
  // The rows p of each front in `parts` workgroups; a row takes at most m columns.
  const int parts = sweep_parts(a.nlevel, a.max_p);
  const int ntl = large_threads(a.nlevel * parts);
  const int rows = (std::max(a.max_p, 1) + parts - 1) / parts;
  const int g = std::max(1, ntl / rows);
  return SweepShape{2, std::max(16, prefetch_depth((a.max_m + g - 1) / g, cap)), ntl, parts};
}

bool sweep_shape_ok(const LevelArgs& a, bool fwd, size_t elem, int nr, const SweepShape& s) {
  if (s.kind == 0) return true;
  if (s.kind == 1) {
    if (!wave_level(a) || s.ntl != 64 || s.parts != 1) return false;
    const int rpl = fwd && a.max_m > 64 ? 2 : 1;
    return (s.kp == 8 || s.kp == 16 || s.kp == 32) && s.kp <= wave_kp_max(elem, rpl);
  }
  if (s.kind != 2) return false;
  if (s.ntl != 256 && s.ntl != 512 && s.ntl != 1024) return false;
  if (s.parts != 1 && s.parts != 2 && s.parts != 4 && s.parts != 8) return false;
  if (s.kp != 16 && s.kp != 32) return false;
  if (s.kp > large_kp_max(elem)) return false;
  if (sweep_lds(a, fwd, elem, nr, s.ntl) > (size_t)max_lds()) return false;
  // Backwards, a part that is one of several never writes the front's own
  // vector, which the other parts read: it must hold its rows in one pass.
  if (!fwd && s.parts > 1 && (a.max_p + s.parts - 1) / s.parts > s.ntl) return false;
  return true;
}

std::vector<SweepShape> sweep_candidates(const LevelArgs& a, bool fwd, size_t elem, int nr) {
  std::vector<SweepShape> out;
  out.push_back(sweep_default(a, fwd, elem));
  auto add = [&](SweepShape s) {
    if (!sweep_shape_ok(a, fwd, elem, nr, s)) return;
    for (const SweepShape& o : out)
      if (o.kind == s.kind && o.kp == s.kp && o.ntl == s.ntl && o.parts == s.parts) return;
    out.push_back(s);
  };
  if (wave_level(a)) {
    for (int kp : {8, 16, 32}) add(SweepShape{1, kp, 64, 1});
    // one workgroup per front for the wider fronts of these levels
    if (a.max_m > 64)
      for (int kp : {16, 32}) add(SweepShape{2, kp, 256, 1});
    return out;
  }
  const int rows = fwd ? a.max_m : std::max(a.max_p, 1);
  for (int parts : {1, 2, 4, 8}) {
    if (parts > 1 && (long long)a.nlevel * parts > 4LL * num_cus()) continue;   // already full
    if (parts > 1 && rows / parts < 16) continue;
    for (int ntl : {256, 512, 1024})
      for (int kp : {16, 32}) add(SweepShape{2, kp, ntl, parts});
  }
  return out;
}

template <typename T>
void launch_sweep_fwd(hipStream_t st, const LevelArgs& a, const T* fac, const int* piv, T* vec,
                      const RhsSet& r, SweepShape sh) {
  check_rhs(r);
  if (sh.kind == 0) sh = sweep_default(a, true, sizeof(T));
  if (!sweep_shape_ok(a, true, sizeof(T), r.nr, sh)) throw Error(STF_EINVAL, "sweep launch shape not valid for the level");
  if (sh.kind == 1) {
    constexpr int K32 = sizeof(T) == 8 ? 32 : 16;
    constexpr int K16R2 = sizeof(T) == 8 ? 16 : 8;
    if (a.max_m <= 64) {
      if (sh.kp == 8) fwd_wave_launch<T, 1, 8>(st, a, fac, piv, vec, r);
      else if (sh.kp == 16) fwd_wave_launch<T, 1, 16>(st, a, fac, piv, vec, r);
      else fwd_wave_launch<T, 1, K32>(st, a, fac, piv, vec, r);
    } else {
      if (sh.kp == 8) fwd_wave_launch<T, 2, 8>(st, a, fac, piv, vec, r);
      else fwd_wave_launch<T, 2, K16R2>(st, a, fac, piv, vec, r);
    }
    return;
  }
  if (sh.ntl == 256) fwd_large_launch<T, 256>(st, a, sh.parts, sh.kp, fac, piv, vec, r);
  else if (sh.ntl == 512) fwd_large_launch<T, 512>(st, a, sh.parts, sh.kp, fac, piv, vec, r);
  else fwd_large_launch<T, 1024>(st, a, sh.parts, sh.kp, fac, piv, vec, r);
}

template <typename T>
void launch_sweep_bwd(hipStream_t st, const LevelArgs& a, const T* upk, T* vec, T* u,
                      const RhsSet& r, SweepShape sh) {
  check_rhs(r);
  if (sh.kind == 0) sh = sweep_default(a, false, sizeof(T));
  if (!sweep_shape_ok(a, false, sizeof(T), r.nr, sh)) throw Error(STF_EINVAL, "sweep launch shape not valid for the level");
  if (sh.kind == 1) {
    constexpr int K32 = sizeof(T) == 8 ? 32 : 16;
    if (sh.kp == 8) bwd_wave_launch<T, 8>(st, a, upk, vec, u, r);
    else if (sh.kp == 16) bwd_wave_launch<T, 16>(st, a, upk, vec, u, r);
    else bwd_wave_launch<T, K32>(st, a, upk, vec, u, r);
    return;
  }
  if (sh.ntl == 256) bwd_large_launch<T, 256>(st, a, sh.parts, sh.kp, upk, vec, u, r);
  else if (sh.ntl == 512) bwd_large_launch<T, 512>(st, a, sh.parts, sh.kp, upk, vec, u, r);
  else bwd_large_launch<T, 1024>(st, a, sh.parts, sh.kp, upk, vec, u, r);
}

// LDS of the subtree sweeps besides the slots: the wavefronts' scratch.
size_t subtree_scratch(size_t elem, int nr, int rpl, bool fwd) {
  return (size_t)4 * nr * (fwd ? 64 * rpl : 128) * elem;
}

bool subtree_ok(const FuseArgs& z, size_t elem, int nr) {
  if (z.K < 1 || z.ntrees < 1 || z.max_m > 128 || z.max_p > 64 || z.slot_q < 0) return false;
  const int rpl = z.max_m <= 64 ? 1 : 2;
  const size_t dyn = (size_t)z.slot_q * nr * elem;
  return dyn + subtree_scratch(elem, nr, rpl, true) <= (size_t)max_lds() &&
         dyn + subtree_scratch(elem, nr, 1, false) <= (size_t)max_lds();
}

template <typename T>
void launch_fwd_subtree(hipStream_t st, const LevelArgs& a, const FuseArgs& z, const T* lpk, const int* piv,
                        T* vec, const RhsSet& r) {
  check_rhs(r);
  if (!subtree_ok(z, sizeof(T), r.nr)) throw Error(STF_EINVAL, "subtree sweep does not fit the levels");
  const size_t lds = (size_t)z.slot_q * r.nr * sizeof(T);
  const int rpl = z.max_m <= 64 ? 1 : 2;
  const int kp = prefetch_depth(z.max_p, 16 / rpl);
#define STF_CALL(NR)                                                                                  \
  if (rpl == 2)                                                                                       \
    STF_LAUNCH((k_fwd_subtree<T, 2, 8, NR>), dim3(z.ntrees), dim3(NT), lds, st, a, z, lpk, piv, \
                       vec, r);                                                                       \
  else if (kp == 8)                                                                                   \
    STF_LAUNCH((k_fwd_subtree<T, 1, 8, NR>), dim3(z.ntrees), dim3(NT), lds, st, a, z, lpk, piv, \
                       vec, r);                                                                       \
  else                                                                                                \
    STF_LAUNCH((k_fwd_subtree<T, 1, 16, NR>), dim3(z.ntrees), dim3(NT), lds, st, a, z, lpk, piv, \
                       vec, r)
  STF_NR_DISPATCH(r.nr, STF_CALL)
#undef STF_CALL
}

template <typename T>
void launch_bwd_subtree(hipStream_t st, const LevelArgs& a, const FuseArgs& z, const T* upk, T* vec, T* u,
                        const RhsSet& r) {
  check_rhs(r);
  if (!subtree_ok(z, sizeof(T), r.nr)) throw Error(STF_EINVAL, "subtree sweep does not fit the levels");
  const size_t lds = (size_t)z.slot_q * r.nr * sizeof(T);
  // Row groups as in the level kernels: W >= max_p lanes, G = 64 / W per row.
  int w = 4;
  while (w < z.max_p) w *= 2;
  const int g = 64 / w;
  const int kp = prefetch_depth((z.max_m + g - 1) / g, 16);
#define STF_CALL(NR)                                                                                   \
  if (kp == 8)                                                                                         \
    STF_LAUNCH((k_bwd_subtree<T, 8, NR>), dim3(z.ntrees), dim3(NT), lds, st, a, z, upk, vec, u, r); \
  else                                                                                                 \
    STF_LAUNCH((k_bwd_subtree<T, 16, NR>), dim3(z.ntrees), dim3(NT), lds, st, a, z, upk, vec, u, r)
  STF_NR_DISPATCH(r.nr, STF_CALL)
#undef STF_CALL
}

template <typename T>
void launch_scatter(hipStream_t st, const T* u, const SubDev* subs, const int4* cover_x,
                    const int4* cover_y, const ScatDev* probs, int nprob, int max_nx, int max_ny,
                    const int* pact, const RhsSet& r) {
  check_rhs(r);
  dim3 blk(64, 4), grd((max_nx + 63) / 64, (max_ny + 3) / 4, nprob);
#define STF_CALL(NR) \
  STF_LAUNCH((k_scatter<T, NR>), grd, blk, 0, st, u, subs, cover_x, cover_y, probs, pact, r)
  STF_NR_DISPATCH(r.nr, STF_CALL)
#undef STF_CALL
}

void launch_stage_residual(hipStream_t st, const double2* keps, const double2* gc,
                           const SubDev* subs, const ScatDev* probs, const int* slist, int sfirst,
                           int scount, int maxw, int maxh, const int* pact, const RhsSet& r,
                           double2* rbuf, long long rstride) {
  check_rhs(r);
  if (scount <= 0) return;
  dim3 blk(64, 4), grd((maxw + 63) / 64, (maxh + 3) / 4, scount);
#define STF_CALL(NR)                                                                            \
  STF_LAUNCH((k_stage_residual<NR>), grd, blk, 0, st, keps, gc, subs, probs, slist, sfirst, \
                     pact, r, rbuf, rstride)
  STF_NR_DISPATCH(r.nr, STF_CALL)
#undef STF_CALL
}

template <typename T>
void launch_stage_scatter(hipStream_t st, const T* u, const SubDev* subs, const ScatDev* probs,
                          const int4* cover_x, const int4* cover_y, const int* slist, int sfirst,
                          int scount, int maxw, int maxh, const int* inst, const int* pact,
                          const RhsSet& r) {
  check_rhs(r);
  if (scount <= 0) return;
  dim3 blk(64, 4), grd((maxw + 63) / 64, (maxh + 3) / 4, scount);
#define STF_CALL(NR)                                                                            \
  STF_LAUNCH((k_stage_scatter<T, NR>), grd, blk, 0, st, u, subs, probs, cover_x, cover_y, \
                     slist, sfirst, inst, pact, r)
  STF_NR_DISPATCH(r.nr, STF_CALL)
#undef STF_CALL
}

template <typename T>
void launch_stage_scatter_first(hipStream_t st, const T* u, const SubDev* subs, const int4* cover_x,
                                const int4* cover_y, const ScatDev* probs, int nprob, int max_nx,
                                int max_ny, const int* inst, const int* pact, const RhsSet& r) {
  check_rhs(r);
  dim3 blk(64, 4), grd((max_nx + 63) / 64, (max_ny + 3) / 4, nprob);
#define STF_CALL(NR)                                                                              \
  STF_LAUNCH((k_stage_scatter_first<T, NR>), grd, blk, 0, st, u, subs, cover_x, cover_y, probs, \
                     inst, pact, r)
  STF_NR_DISPATCH(r.nr, STF_CALL)
#undef STF_CALL
}

void launch_zero(hipStream_t st, double2* p, long long n) {
  long long g = (n + 255) / 256;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  STF_LAUNCH(k_zero, dim3((unsigned)g), dim3(256), 0, st, p, n);
}

template <typename T>
void launch_overlap_norm(hipStream_t st, const T* u, const SubDev* subs, int nsub, double* per_sub,
                         double* out) {
  STF_LAUNCH((k_overlap_norm<T>), dim3(nsub), dim3(256), 0, st, u, subs, per_sub);
  STF_LAUNCH(k_sum_ordered, dim3(1), dim3(64), 0, st, per_sub, nsub, out);
}

#define STF_INST(T)                                                                             \
  template void launch_front_factor<T>(hipStream_t, const LevelArgs&, T*, T*, T*, int*, int*, double, \
                                       FactorShape);                                            \
  template void launch_sweep_fwd<T>(hipStream_t, const LevelArgs&, const T*, const int*, T*,    \
                                    const RhsSet&, SweepShape);                                 \
  template void launch_sweep_bwd<T>(hipStream_t, const LevelArgs&, const T*, T*, T*,            \
                                    const RhsSet&, SweepShape);                                 \
  template void launch_fwd_subtree<T>(hipStream_t, const LevelArgs&, const FuseArgs&, const T*, \
                                      const int*, T*, const RhsSet&);                           \
  template void launch_bwd_subtree<T>(hipStream_t, const LevelArgs&, const FuseArgs&, const T*, \
                                      T*, T*, const RhsSet&);                                   \
  template void launch_scatter<T>(hipStream_t, const T*, const SubDev*, const int4*,            \
                                  const int4*, const ScatDev*, int, int, int, const int*,       \
                                  const RhsSet&);                                               \
  template void launch_overlap_norm<T>(hipStream_t, const T*, const SubDev*, int, double*,      \
                                       double*);                                                \
  template void launch_stage_scatter<T>(hipStream_t, const T*, const SubDev*, const ScatDev*,   \
                                        const int4*, const int4*, const int*, int, int, int, int,\
                                        const int*, const int*, const RhsSet&);                 \
  template void launch_stage_scatter_first<T>(hipStream_t, const T*, const SubDev*, const int4*, \
                                              const int4*, const ScatDev*, int, int, int,        \
                                              const int*, const int*, const RhsSet&);
STF_INST(double2)
STF_INST(float2)

}  // namespace stf
