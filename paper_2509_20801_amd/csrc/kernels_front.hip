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
// summed rows; swaps are applied to whole rows and recorded LAPACK-style
// (piv[k] = row exchanged with row k at step k, front-relative).
//
// Front vectors: each front owns m entries at vec_off.  The forward sweep
// leaves [y_p ; update contribution] there, the backward sweep [x_p ; x_q],
// from which the children gather their x_q.  Every write has one owner, so the
// sweeps are deterministic without atomics.
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
constexpr int WB = 64;         // diagonal block (one wavefront) of the large sweeps
constexpr int PF = 8;          // columns prefetched per chunk in the wave sweeps
constexpr int UC = 32;         // columns of U staged in LDS per trailing-update chunk

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

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
      double2 ke = a.keps[(long long)(s.oy0 + ty) * a.nx + (s.ox0 + tx)];
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
  for (int ci = 0; ci < f.nchild; ++ci) {
    const FrontDev cf = a.fronts[a.children[f.child_off + ci]];
    const int mc = cf.p + cf.q, q = cf.q;
    const T* S = fac + cf.fac_off + (long long)cf.p * mc + cf.p;   // F22 of the child
    const int* cm = a.cmap + cf.cmap_off;
    const long long qq = (long long)q * q;
    for (long long t = tid; t < qq; t += nthr) {
      int j = (int)(t / q), i = (int)(t - (long long)j * q);        // (i, j) of S, i fastest
      T v = S[(long long)j * mc + i];
      T* d = G + (long long)cm[j] * m + cm[i];
      *d = cadd(*d, v);
    }
    sync();
  }
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

// ---------------------------------------------------------------------------
// Factorisation, small fronts: one wavefront per front, front in LDS.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(64) void k_factor_small(LevelArgs a, T* __restrict__ fac,
                                                     int* __restrict__ piv, int* __restrict__ flag,
                                                     double tau) {
  using R = typename RealOf<T>::type;
  extern __shared__ unsigned char smem_raw[];
  T* G = reinterpret_cast<T*>(smem_raw);
  const FrontDev f = a.fronts[a.level_list[blockIdx.x]];
  const int m = f.p + f.q, p = f.p, lane = threadIdx.x;
  assemble_front<T>(a, fac, f, G, lane, 64, [] { wave_sync(); });
  int* ip = piv + f.piv_off;
  for (int k = 0; k < p; ++k) {
    int bi;
    R best, amax;
    wave_pivot(G + (long long)k * m, k, p, m, lane, bi, best, amax);
    if (lane == 0) {
      T v = G[(long long)k * m + bi];
      if (perturb(v, best, amax, tau)) {
        G[(long long)k * m + bi] = v;
        atomicOr(flag, 1);
      }
      ip[k] = bi;
    }
    wave_sync();
    if (bi != k)
      for (int c = lane; c < m; c += 64) {
        T t0 = G[(long long)c * m + k];
        G[(long long)c * m + k] = G[(long long)c * m + bi];
        G[(long long)c * m + bi] = t0;
      }
    wave_sync();
    const T dinv = cdiv(T{(R)1, (R)0}, G[(long long)k * m + k]);
    for (int r = k + 1 + lane; r < m; r += 64) {
      T l = cmul(G[(long long)k * m + r], dinv);
      G[(long long)k * m + r] = l;
      for (int c = k + 1; c < m; ++c)
        G[(long long)c * m + r] = cfms(l, G[(long long)c * m + k], G[(long long)c * m + r]);
    }
    wave_sync();
  }
  T* F = fac + f.fac_off;
  const long long mm = (long long)m * m;
  for (long long t = lane; t < mm; t += 64) F[t] = G[t];
}

// ---------------------------------------------------------------------------
// Factorisation, large fronts: one 256-thread workgroup per front.  Assembly in
// global memory, then blocked right-looking LU: a panel of NB columns is
// factored in LDS by one wavefront, U12 is solved one column per thread and
// the trailing matrix is updated with each thread owning one row (its NB
// multipliers in registers) against U columns staged in LDS.
// ---------------------------------------------------------------------------
template <typename T, int NB>
__global__ __launch_bounds__(NT) void k_factor_large(LevelArgs a, T* __restrict__ fac,
                                                     int* __restrict__ piv, int* __restrict__ flag,
                                                     double tau) {
  using R = typename RealOf<T>::type;
  extern __shared__ unsigned char smem_raw[];
  T* P = reinterpret_cast<T*>(smem_raw);           // panel, column-major, ld = ldp
  __shared__ T Us[UC][NB + 1];                      // staged U columns
  __shared__ int s_piv[NB];
  const FrontDev f = a.fronts[a.level_list[blockIdx.x]];
  const int m = f.p + f.q, p = f.p, ldp = a.max_m;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  T* F = fac + f.fac_off;
  assemble_front<T>(a, fac, f, F, tid, NT, [] { __syncthreads(); });
  int* ip = piv + f.piv_off;

  for (int kb = 0; kb < p; kb += NB) {
    const int nb = min(NB, p - kb);
    const int nr = m - kb;
    for (int t = tid; t < nb * nr; t += NT) {
      int k = t / nr, r = t - k * nr;
      P[k * ldp + r] = F[(long long)(kb + k) * m + kb + r];
    }
    __syncthreads();
    if (wv == 0) {
      for (int k = 0; k < nb; ++k) {
        T* col = P + k * ldp;
        int bi;
        R best, amax;
        wave_pivot(col, k, p - kb, nr, lane, bi, best, amax);
        if (lane == 0) {
          T v = col[bi];
          if (perturb(v, best, amax, tau)) {
            col[bi] = v;
            atomicOr(flag, 1);
          }
          s_piv[k] = bi;
          ip[kb + k] = kb + bi;
        }
        wave_sync();
        if (bi != k && lane < nb) {
          T t0 = P[lane * ldp + k];
          P[lane * ldp + k] = P[lane * ldp + bi];
          P[lane * ldp + bi] = t0;
        }
        wave_sync();
        const T dinv = cdiv(T{(R)1, (R)0}, col[k]);
        for (int r = k + 1 + lane; r < nr; r += 64) {
          T l = cmul(col[r], dinv);
          col[r] = l;
          for (int c = k + 1; c < nb; ++c) P[c * ldp + r] = cfms(l, P[c * ldp + k], P[c * ldp + r]);
        }
        wave_sync();
      }
    }
    __syncthreads();
    for (int t = tid; t < nb * nr; t += NT) {
      int k = t / nr, r = t - k * nr;
      F[(long long)(kb + k) * m + kb + r] = P[k * ldp + r];
    }
    // Row exchanges in the columns outside the panel, in pivot order.
    for (int c = tid; c < m; c += NT) {
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
    for (int c = kb + nb + tid; c < m; c += NT) {
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
    // Trailing update over rows/cols n0 .. m-1.
    const int n0 = kb + nb;
    for (int r0 = n0; r0 < m; r0 += NT) {
      const int r = r0 + tid;
      T lr[NB];
#pragma unroll
      for (int t = 0; t < NB; ++t) lr[t] = (t < nb && r < m) ? P[t * ldp + (r - kb)] : czero<T>();
      for (int c0 = n0; c0 < m; c0 += UC) {
        const int cw = min(UC, m - c0);
        __syncthreads();
        for (int t = tid; t < cw * NB; t += NT) {
          int c = t / NB, k = t - c * NB;
          Us[c][k] = (k < nb) ? F[(long long)(c0 + c) * m + kb + k] : czero<T>();
        }
        __syncthreads();
        if (r < m) {
          for (int c = 0; c < cw; ++c) {
            T* dst = F + (long long)(c0 + c) * m + r;
            T acc = *dst;
#pragma unroll
            for (int t = 0; t < NB; ++t) acc = cfms(lr[t], Us[c][t], acc);
            *dst = acc;
          }
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Sweeps, small fronts (m <= 64): one wavefront per front, lane = row.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(64) void k_fwd_small(LevelArgs a, const T* __restrict__ fac,
                                                  const int* __restrict__ piv, T* __restrict__ vec,
                                                  const double2* __restrict__ v) {
  __shared__ T vl[64];
  const FrontDev f = a.fronts[a.level_list[blockIdx.x]];
  const int m = f.p + f.q, p = f.p, lane = threadIdx.x;
  const T* F = fac + f.fac_off;
  T val = czero<T>();
  if (lane < p) {
    const SubDev s = a.subs[f.sub];
    int node = a.vars[f.var_off + lane];
    int gx = s.ox0 + node % s.nxl, gy = s.oy0 + node / s.nxl;
    if (gx >= s.ix0 && gx < s.ix1 && gy >= s.iy0 && gy < s.iy1)
      val = from_d2<T>(v[(long long)gy * a.nx + gx]);
  }
  vl[lane] = val;
  wave_sync();
  for (int ci = 0; ci < f.nchild; ++ci) {
    const FrontDev cf = a.fronts[a.children[f.child_off + ci]];
    if (lane < cf.q) {
      int dst = a.cmap[cf.cmap_off + lane];
      vl[dst] = cadd(vl[dst], vec[cf.vec_off + cf.p + lane]);
    }
    wave_sync();
  }
  if (lane == 0) {
    const int* ip = piv + f.piv_off;
    for (int k = 0; k < p; ++k) {
      int r2 = ip[k];
      if (r2 != k) { T t0 = vl[k]; vl[k] = vl[r2]; vl[r2] = t0; }
    }
  }
  wave_sync();
  val = vl[lane];
  const bool row = lane < m;
  for (int k0 = 0; k0 < p; k0 += PF) {
    T col[PF];
#pragma unroll
    for (int t = 0; t < PF; ++t)
      col[t] = (row && k0 + t < p) ? F[(long long)(k0 + t) * m + lane] : czero<T>();
#pragma unroll
    for (int t = 0; t < PF; ++t) {
      const int k = k0 + t;
      if (k < p) {
        T yk = shfl_c(val, k);
        if (lane > k) val = cfms(col[t], yk, val);
      }
    }
  }
  if (row) vec[f.vec_off + lane] = val;
}

template <typename T>
__global__ __launch_bounds__(64) void k_bwd_small(LevelArgs a, const T* __restrict__ fac,
                                                  T* __restrict__ vec, T* __restrict__ u) {
  const FrontDev f = a.fronts[a.level_list[blockIdx.x]];
  const int m = f.p + f.q, p = f.p, lane = threadIdx.x;
  const T* F = fac + f.fac_off;
  T val = czero<T>();
  if (lane < p) {
    val = vec[f.vec_off + lane];
  } else if (lane < m) {
    const FrontDev pf = a.fronts[f.parent];
    val = vec[pf.vec_off + a.cmap[f.cmap_off + lane - p]];
  }
  // y - U12 x_q
  for (int j0 = p; j0 < m; j0 += PF) {
    T col[PF];
#pragma unroll
    for (int t = 0; t < PF; ++t)
      col[t] = (lane < p && j0 + t < m) ? F[(long long)(j0 + t) * m + lane] : czero<T>();
#pragma unroll
    for (int t = 0; t < PF; ++t) {
      const int j = j0 + t;
      if (j < m) {
        T xj = shfl_c(val, j);
        if (lane < p) val = cfms(col[t], xj, val);
      }
    }
  }
  // U11 x = y'
  for (int k1 = p; k1 > 0; k1 -= PF) {
    T col[PF];
#pragma unroll
    for (int t = 0; t < PF; ++t) {
      const int k = k1 - 1 - t;
      col[t] = (k >= 0 && lane <= k) ? F[(long long)k * m + lane] : czero<T>();
    }
#pragma unroll
    for (int t = 0; t < PF; ++t) {
      const int k = k1 - 1 - t;
      if (k >= 0) {
        T xk = (lane == k) ? cdiv(val, col[t]) : val;
        xk = shfl_c(xk, k);
        if (lane == k) val = xk;
        else if (lane < k) val = cfms(col[t], xk, val);
      }
    }
  }
  if (lane < m) vec[f.vec_off + lane] = val;
  if (lane < p) {
    const SubDev s = a.subs[f.sub];
    u[s.u_off + a.vars[f.var_off + lane]] = val;
  }
}

// ---------------------------------------------------------------------------
// Sweeps, large fronts: one workgroup per front; diagonal blocks of 64 columns
// solved by wavefront 0, the rest of each column block applied by all threads
// (one row per thread, column-block GEMV with coalesced column reads).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(NT) void k_fwd_large(LevelArgs a, const T* __restrict__ fac,
                                                  const int* __restrict__ piv, T* __restrict__ vec,
                                                  const double2* __restrict__ v) {
  extern __shared__ unsigned char smem_raw[];
  T* vl = reinterpret_cast<T*>(smem_raw);
  const FrontDev f = a.fronts[a.level_list[blockIdx.x]];
  const int m = f.p + f.q, p = f.p;
  const T* F = fac + f.fac_off;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const SubDev s = a.subs[f.sub];
  for (int i = tid; i < m; i += NT) {
    T val = czero<T>();
    if (i < p) {
      int node = a.vars[f.var_off + i];
      int gx = s.ox0 + node % s.nxl, gy = s.oy0 + node / s.nxl;
      if (gx >= s.ix0 && gx < s.ix1 && gy >= s.iy0 && gy < s.iy1)
        val = from_d2<T>(v[(long long)gy * a.nx + gx]);
    }
    vl[i] = val;
  }
  __syncthreads();
  for (int ci = 0; ci < f.nchild; ++ci) {
    const FrontDev cf = a.fronts[a.children[f.child_off + ci]];
    const int* cm = a.cmap + cf.cmap_off;
    const T* cv = vec + cf.vec_off + cf.p;
    for (int i = tid; i < cf.q; i += NT) vl[cm[i]] = cadd(vl[cm[i]], cv[i]);
    __syncthreads();
  }
  if (tid == 0) {
    const int* ip = piv + f.piv_off;
    for (int k = 0; k < p; ++k) {
      int r2 = ip[k];
      if (r2 != k) { T t0 = vl[k]; vl[k] = vl[r2]; vl[r2] = t0; }
    }
  }
  __syncthreads();
  for (int kb = 0; kb < p; kb += WB) {
    const int nbk = min(WB, p - kb);
    if (wv == 0) {
      T val = lane < nbk ? vl[kb + lane] : czero<T>();
      for (int k0 = 0; k0 < nbk; k0 += PF) {
        T col[PF];
#pragma unroll
        for (int t = 0; t < PF; ++t)
          col[t] = (lane < nbk && k0 + t < nbk) ? F[(long long)(kb + k0 + t) * m + kb + lane]
                                                : czero<T>();
#pragma unroll
        for (int t = 0; t < PF; ++t) {
          const int k = k0 + t;
          if (k < nbk) {
            T yk = shfl_c(val, k);
            if (lane > k) val = cfms(col[t], yk, val);
          }
        }
      }
      if (lane < nbk) vl[kb + lane] = val;
    }
    __syncthreads();
    for (int r = kb + nbk + tid; r < m; r += NT) {
      T acc = czero<T>();
      const T* Fr = F + (long long)kb * m + r;
      for (int k = 0; k < nbk; ++k) acc = cfma(Fr[(long long)k * m], vl[kb + k], acc);
      vl[r] = csub(vl[r], acc);
    }
    __syncthreads();
  }
  T* out = vec + f.vec_off;
  for (int i = tid; i < m; i += NT) out[i] = vl[i];
}

template <typename T>
__global__ __launch_bounds__(NT) void k_bwd_large(LevelArgs a, const T* __restrict__ fac,
                                                  T* __restrict__ vec, T* __restrict__ u) {
  extern __shared__ unsigned char smem_raw[];
  T* vl = reinterpret_cast<T*>(smem_raw);
  const FrontDev f = a.fronts[a.level_list[blockIdx.x]];
  const int m = f.p + f.q, p = f.p;
  const T* F = fac + f.fac_off;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  T* fv = vec + f.vec_off;
  for (int i = tid; i < p; i += NT) vl[i] = fv[i];
  if (f.parent >= 0) {
    const FrontDev pf = a.fronts[f.parent];
    const int* cm = a.cmap + f.cmap_off;
    const T* pv = vec + pf.vec_off;
    for (int i = tid; i < f.q; i += NT) vl[p + i] = pv[cm[i]];
  }
  __syncthreads();
  // y - U12 x_q, one row per thread.
  for (int r = tid; r < p; r += NT) {
    T acc = czero<T>();
    const T* Fr = F + r;
    for (int j = p; j < m; ++j) acc = cfma(Fr[(long long)j * m], vl[j], acc);
    vl[r] = csub(vl[r], acc);
  }
  __syncthreads();
  for (int kb = ((p - 1) / WB) * WB; kb >= 0; kb -= WB) {
    const int nbk = min(WB, p - kb);
    if (wv == 0) {
      T val = lane < nbk ? vl[kb + lane] : czero<T>();
      for (int k1 = nbk; k1 > 0; k1 -= PF) {
        T col[PF];
#pragma unroll
        for (int t = 0; t < PF; ++t) {
          const int k = k1 - 1 - t;
          col[t] = (k >= 0 && lane <= k) ? F[(long long)(kb + k) * m + kb + lane] : czero<T>();
        }
#pragma unroll
        for (int t = 0; t < PF; ++t) {
          const int k = k1 - 1 - t;
          if (k >= 0) {
            T xk = (lane == k) ? cdiv(val, col[t]) : val;
            xk = shfl_c(xk, k);
            if (lane == k) val = xk;
            else if (lane < k) val = cfms(col[t], xk, val);
          }
        }
      }
      if (lane < nbk) vl[kb + lane] = val;
    }
    __syncthreads();
    for (int r = tid; r < kb; r += NT) {
      T acc = czero<T>();
      const T* Fr = F + (long long)kb * m + r;
      for (int k = 0; k < nbk; ++k) acc = cfma(Fr[(long long)k * m], vl[kb + k], acc);
      vl[r] = csub(vl[r], acc);
    }
    __syncthreads();
  }
  const int* vars = a.vars + f.var_off;
  const long long uo = a.subs[f.sub].u_off;
  for (int i = tid; i < m; i += NT) {
    fv[i] = vl[i];
    if (i < p) u[uo + vars[i]] = vl[i];
  }
}

// z = sum_k P_k u_k: each global node adds the local fields of the (at most
// four) subdomains whose Omega_k covers it, in a fixed order.
template <typename T>
__global__ __launch_bounds__(256) void k_scatter(const T* __restrict__ u, const SubDev* __restrict__ subs,
                                                 const int4* __restrict__ cover_x,
                                                 const int4* __restrict__ cover_y, int px, int nx,
                                                 int ny, double2* __restrict__ z) {
  int i = blockIdx.x * 64 + threadIdx.x;
  int j = blockIdx.y * 4 + threadIdx.y;
  if (i >= nx || j >= ny) return;
  int4 cx = cover_x[i], cy = cover_y[j];
  double2 acc = make_double2(0.0, 0.0);
  int kys[2] = {cy.x, cy.z}, uys[2] = {cy.y, cy.w};
  int kxs[2] = {cx.x, cx.z}, txs[2] = {cx.y, cx.w};
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    if (kys[b] < 0) continue;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      if (kxs[c] < 0) continue;
      const SubDev& s = subs[kys[b] * px + kxs[c]];
      double2 val = to_d2(u[s.u_off + (long long)uys[b] * s.nxl + txs[c]]);
      acc.x += val.x;
      acc.y += val.y;
    }
  }
  z[(long long)j * nx + i] = acc;
}

int g_max_lds = 0;
int max_lds() {
  if (g_max_lds == 0) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
        v > 0)
      g_max_lds = std::min(v, 65536);
    else
      g_max_lds = 65536;
  }
  return g_max_lds;
}

template <typename T, int NB>
void large_launch(hipStream_t st, const LevelArgs& a, T* fac, int* piv, int* flag, double tau) {
  size_t lds = (size_t)a.max_m * NB * sizeof(T);
  hipLaunchKernelGGL((k_factor_large<T, NB>), dim3(a.nlevel), dim3(NT), lds, st, a, fac, piv, flag,
                     tau);
}

}  // namespace

int small_factor_limit(size_t elem) {
  // Largest front order whose m x m block fits the LDS of one wavefront workgroup.
  int lim = 1;
  while ((size_t)(lim + 1) * (lim + 1) * elem <= 32768) ++lim;
  return std::min(lim, 64);
}

template <typename T>
void launch_front_factor(hipStream_t st, const LevelArgs& a, T* fac, int* piv, int* flag,
                         double tau) {
  if (a.max_m <= small_factor_limit(sizeof(T))) {
    size_t lds = (size_t)a.max_m * a.max_m * sizeof(T);
    hipLaunchKernelGGL(k_factor_small<T>, dim3(a.nlevel), dim3(64), lds, st, a, fac, piv, flag, tau);
    return;
  }
  // Panel width: as wide as the LDS allows for the largest front of the level
  // (the staged U chunk and small arrays take the rest).
  const size_t budget = (size_t)max_lds() - (size_t)UC * 33 * sizeof(T) - 512;
  const size_t per_col = (size_t)a.max_m * sizeof(T);
  const int nb_max = sizeof(T) == 16 ? 16 : 32;
  int nb = 1;
  while (nb * 2 <= nb_max && per_col * nb * 2 <= budget) nb *= 2;
  if (per_col * nb > budget) throw Error(STF_EINVAL, "front too large for the LDS panel");
  switch (nb) {
    case 32: large_launch<T, 32>(st, a, fac, piv, flag, tau); break;
    case 16: large_launch<T, 16>(st, a, fac, piv, flag, tau); break;
    case 8: large_launch<T, 8>(st, a, fac, piv, flag, tau); break;
    case 4: large_launch<T, 4>(st, a, fac, piv, flag, tau); break;
    case 2: large_launch<T, 2>(st, a, fac, piv, flag, tau); break;
    default: large_launch<T, 1>(st, a, fac, piv, flag, tau); break;
  }
}

template <typename T>
void launch_sweep_fwd(hipStream_t st, const LevelArgs& a, const T* fac, const int* piv, T* vec,
                      const double2* v) {
  if (a.max_m <= 64) {
    hipLaunchKernelGGL(k_fwd_small<T>, dim3(a.nlevel), dim3(64), 0, st, a, fac, piv, vec, v);
  } else {
    size_t lds = (size_t)a.max_m * sizeof(T);
    hipLaunchKernelGGL(k_fwd_large<T>, dim3(a.nlevel), dim3(NT), lds, st, a, fac, piv, vec, v);
  }
}

template <typename T>
void launch_sweep_bwd(hipStream_t st, const LevelArgs& a, const T* fac, T* vec, T* u) {
  if (a.max_m <= 64) {
    hipLaunchKernelGGL(k_bwd_small<T>, dim3(a.nlevel), dim3(64), 0, st, a, fac, vec, u);
  } else {
    size_t lds = (size_t)a.max_m * sizeof(T);
    hipLaunchKernelGGL(k_bwd_large<T>, dim3(a.nlevel), dim3(NT), lds, st, a, fac, vec, u);
  }
}

template <typename T>
void launch_scatter(hipStream_t st, const T* u, const SubDev* subs, const int4* cover_x,
                    const int4* cover_y, int px, int nx, int ny, double2* z) {
  dim3 blk(64, 4), grd((nx + 63) / 64, (ny + 3) / 4);
  hipLaunchKernelGGL(k_scatter<T>, grd, blk, 0, st, u, subs, cover_x, cover_y, px, nx, ny, z);
}

#define STF_INST(T)                                                                             \
  template void launch_front_factor<T>(hipStream_t, const LevelArgs&, T*, int*, int*, double);  \
  template void launch_sweep_fwd<T>(hipStream_t, const LevelArgs&, const T*, const int*, T*,    \
                                    const double2*);                                            \
  template void launch_sweep_bwd<T>(hipStream_t, const LevelArgs&, const T*, T*, T*);           \
  template void launch_scatter<T>(hipStream_t, const T*, const SubDev*, const int4*,            \
                                  const int4*, int, int, int, double2*);
STF_INST(double2)
STF_INST(float2)

}  // namespace stf
