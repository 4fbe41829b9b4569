// Multifrontal LU of the subdomain operators (Sec. 2.4, Eq. (22)) and the
// front sweeps of the local solves (Eq. (23)), batched over every front of one
// elimination-tree level across all subdomains; T = double2 (complex128) or
// float2 (complex64).
//
// Storage: front f of order m = p + q is an m x m row-major block at fac_off:
//   [F11 F12; F21 F22] with the p separator (fully summed) variables first.
// After factorisation F11 holds L11 (unit lower, implicit 1) and U11, F12 holds
// U12, F21 holds L21 and F22 the Schur complement handed to the parent by
// extend-add.  Pivoting is partial, restricted to the p fully summed rows;
// the swaps are applied to whole rows and recorded LAPACK-style (piv[k] = row
// exchanged with row k at step k, front-relative).
//
// Front vectors: each front owns m entries at vec_off.  The forward sweep
// leaves [y_p ; update contribution] there, the backward sweep [x_p ; x_q],
// from which the children gather their x_q.  Every write has one owner, so the
// sweeps are deterministic without atomics.
#include <algorithm>

#include "cplx.h"
#include "stf_internal.h"

namespace stf {

namespace {

constexpr int NT = 256;     // threads per workgroup (4 wavefronts)
constexpr int DB = 32;      // diagonal block of the triangular sweeps

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

template <typename T>
__global__ __launch_bounds__(NT) void k_front_assemble(LevelArgs a, T* __restrict__ fac) {
  const FrontDev f = a.fronts[a.level_list[blockIdx.x]];
  const int m = f.p + f.q;
  T* F = fac + f.fac_off;
  const long long mm = (long long)m * m;
  for (long long t = threadIdx.x; t < mm; t += NT) F[t] = czero<T>();
  __syncthreads();
  const SubDev s = a.subs[f.sub];
  for (int t = threadIdx.x; t < f.ent_cnt; t += NT) {
    SymEntry e = a.ents[f.ent_off + t];
    int r = e.rc & 0xffff, c = (e.rc >> 16) & 0xffff;
    F[(long long)r * m + c] = from_d2<T>(local_coef(a, s, e.nd >> 3, e.nd & 7));
  }
  __syncthreads();
  // Extend-add of the children's Schur complements (one child at a time: two
  // children may update the same entry).
  for (int ci = 0; ci < f.nchild; ++ci) {
    const FrontDev cf = a.fronts[a.children[f.child_off + ci]];
    const int mc = cf.p + cf.q, q = cf.q;
    const T* S = fac + cf.fac_off + (long long)cf.p * mc + cf.p;
    const int* cm = a.cmap + cf.cmap_off;
    const long long qq = (long long)q * q;
    for (long long t = threadIdx.x; t < qq; t += NT) {
      int i = (int)(t / q), j = (int)(t - (long long)i * q);
      T v = S[(long long)i * mc + j];
      T* d = F + (long long)cm[i] * m + cm[j];
      *d = cadd(*d, v);
    }
    __syncthreads();
  }
}

// Blocked right-looking partial LU of one front per workgroup.  The current
// panel (rows kb..m-1, NB columns) is factored in LDS; the U12 block row and
// the trailing matrix are updated in place in global memory (L2-resident for
// the fronts of one level).
template <typename T, int NB>
__global__ __launch_bounds__(NT) void k_front_lu(LevelArgs a, T* __restrict__ fac,
                                                 int* __restrict__ piv, int* __restrict__ flag,
                                                 double tau) {
  using R = typename RealOf<T>::type;
  extern __shared__ unsigned char smem_raw[];
  T* P = reinterpret_cast<T*>(smem_raw);   // panel, row-major with NB columns
  __shared__ R s_best[4], s_amax[4];
  __shared__ int s_bi[4], s_piv;

  const FrontDev f = a.fronts[a.level_list[blockIdx.x]];
  const int m = f.p + f.q, p = f.p;
  T* F = fac + f.fac_off;
  int* ip = piv + f.piv_off;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;

  for (int kb = 0; kb < p; kb += NB) {
    const int nb = min(NB, p - kb);
    const int nr = m - kb;
    for (int t = tid; t < nr * NB; t += NT) {
      int r = t / NB, k = t - r * NB;
      P[t] = (k < nb) ? F[(long long)(kb + r) * m + kb + k] : czero<T>();
    }
    __syncthreads();
    for (int k = 0; k < nb; ++k) {
      // Pivot: largest |.| among the fully summed rows k .. p-kb-1 (ties: lowest row).
      R best = (R)-1, amax = (R)0;
      int bi = k;
      for (int r = k + tid; r < nr; r += NT) {
        R v = cabs2(P[r * NB + k]);
        amax = v > amax ? v : amax;
        if (r < p - kb && v > best) { best = v; bi = r; }
      }
      for (int o = 32; o > 0; o >>= 1) {
        R ob = __shfl_xor(best, o, 64);
        int oi = __shfl_xor(bi, o, 64);
        R oa = __shfl_xor(amax, o, 64);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
        amax = oa > amax ? oa : amax;
      }
      if (lane == 0) { s_best[wv] = best; s_bi[wv] = bi; s_amax[wv] = amax; }
      __syncthreads();
      if (tid == 0) {
        R b0 = s_best[0], am = s_amax[0];
        int i0 = s_bi[0];
        for (int w = 1; w < 4; ++w) {
          if (s_best[w] > b0 || (s_best[w] == b0 && s_bi[w] < i0)) { b0 = s_best[w]; i0 = s_bi[w]; }
          am = s_amax[w] > am ? s_amax[w] : am;
        }
        // Static perturbation of a tiny pivot (reported through *flag).
        R thr = (R)tau * sqrt(am);
        if (!(sqrt(b0) > thr) || b0 <= (R)0) {
          T v = P[i0 * NB + k];
          R mag = sqrt(cabs2(v));
          R tgt = thr > (R)0 ? thr : (R)1e-30;
          P[i0 * NB + k] = mag > (R)0 ? T{v.x / mag * tgt, v.y / mag * tgt} : T{tgt, (R)0};
          atomicOr(flag, 1);
        }
        s_piv = i0;
        ip[kb + k] = kb + i0;
      }
      __syncthreads();
      const int pr = s_piv;
      if (pr != k && tid < NB) {
        T t0 = P[k * NB + tid];
        P[k * NB + tid] = P[pr * NB + tid];
        P[pr * NB + tid] = t0;
      }
      __syncthreads();
      const T dinv = cdiv(T{(R)1, (R)0}, P[k * NB + k]);
      for (int r = k + 1 + tid; r < nr; r += NT) {
        T l = cmul(P[r * NB + k], dinv);
        P[r * NB + k] = l;
#pragma unroll
        for (int c = 1; c < NB; ++c)
          if (k + c < nb) P[r * NB + k + c] = cfms(l, P[k * NB + k + c], P[r * NB + k + c]);
      }
      __syncthreads();
    }
    // Panel back to global memory.
    for (int t = tid; t < nr * NB; t += NT) {
      int r = t / NB, k = t - r * NB;
      if (k < nb) F[(long long)(kb + r) * m + kb + k] = P[t];
    }
    // Row exchanges outside the panel, in pivot order, one column per thread.
    for (int c = tid; c < m; c += NT) {
      if (c >= kb && c < kb + nb) continue;
      for (int k = 0; k < nb; ++k) {
        int r2 = ip[kb + k];
        if (r2 != kb + k) {
          T t0 = F[(long long)(kb + k) * m + c];
          F[(long long)(kb + k) * m + c] = F[(long long)r2 * m + c];
          F[(long long)r2 * m + c] = t0;
        }
      }
    }
    __syncthreads();
    // U12 block row: L_d^{-1} F[kb:kb+nb, kb+nb:m], one column per thread.
    for (int c = kb + nb + tid; c < m; c += NT) {
      T x[NB];
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        if (i < nb) {
          T v = F[(long long)(kb + i) * m + c];
#pragma unroll
          for (int t = 0; t < NB; ++t)
            if (t < i) v = cfms(P[i * NB + t], x[t], v);
          x[i] = v;
          F[(long long)(kb + i) * m + c] = v;
        }
      }
    }
    __syncthreads();
    // Trailing update F22' -= L_panel * U_block over rows/cols kb+nb .. m-1.
    const int n0 = kb + nb, nt = m - n0;
    if (nt > 0) {
      int gw = ((nt < NT ? nt : NT) + 63) / 64 * 64;   // threads per row group
      int ng = NT / gw;                                  // row groups
      int g = tid / gw, lt = tid - g * gw;
      if (g < ng) {
        for (int c = n0 + lt; c < m; c += gw) {
          T u[NB];
#pragma unroll
          for (int t = 0; t < NB; ++t) u[t] = (t < nb) ? F[(long long)(kb + t) * m + c] : czero<T>();
          for (int r = n0 + g; r < m; r += ng) {
            const T* Lr = P + (r - kb) * NB;
            T acc = F[(long long)r * m + c];
#pragma unroll
            for (int t = 0; t < NB; ++t)
              if (t < nb) acc = cfms(Lr[t], u[t], acc);
            F[(long long)r * m + c] = acc;
          }
        }
      }
    }
    __syncthreads();
  }
}

// acc over a row segment, one wavefront per row: returns sum_t row[t]*v[t].
template <typename T>
__device__ inline T wave_dot(const T* __restrict__ row, const T* v, int len, int lane) {
  T acc = czero<T>();
  for (int t = lane; t < len; t += 64) acc = cfma(row[t], v[t], acc);
  return wave_csum(acc);
}

template <typename T>
__global__ __launch_bounds__(NT) void k_sweep_fwd(LevelArgs a, const T* __restrict__ fac,
                                                  const int* __restrict__ piv, T* __restrict__ vec,
                                                  const double2* __restrict__ v) {
  extern __shared__ unsigned char smem_raw[];
  T* vl = reinterpret_cast<T*>(smem_raw);                 // m entries
  __shared__ T Ld[DB][DB + 1];
  const FrontDev f = a.fronts[a.level_list[blockIdx.x]];
  const int m = f.p + f.q, p = f.p;
  const T* F = fac + f.fac_off;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const SubDev s = a.subs[f.sub];
  const int* vars = a.vars + f.var_off;
  // Own source: v restricted to I_k (R_k^I), zero on the extension.
  for (int i = tid; i < m; i += NT) {
    T val = czero<T>();
    if (i < p) {
      int node = vars[i];
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
  // L11 y = P b, by diagonal blocks of DB rows.
  for (int kb = 0; kb < p; kb += DB) {
    const int nbk = min(DB, p - kb);
    for (int r = kb + wv; r < kb + nbk; r += 4) {
      T d = wave_dot(F + (long long)r * m, vl, kb, lane);
      if (lane == 0) vl[r] = csub(vl[r], d);
    }
    for (int t = tid; t < DB * DB; t += NT) {
      int i = t / DB, j = t - i * DB;
      if (i < nbk && j < nbk) Ld[i][j] = F[(long long)(kb + i) * m + kb + j];
    }
    __syncthreads();
    if (wv == 0) {
      T val = lane < nbk ? vl[kb + lane] : czero<T>();
      for (int k = 0; k < nbk; ++k) {
        T yk = shfl_c(val, k);
        if (lane > k && lane < nbk) val = cfms(Ld[lane][k], yk, val);
      }
      if (lane < nbk) vl[kb + lane] = val;
    }
    __syncthreads();
  }
  // Update part: b_q -= L21 y.
  for (int r = p + wv; r < m; r += 4) {
    T d = wave_dot(F + (long long)r * m, vl, p, lane);
    if (lane == 0) vl[r] = csub(vl[r], d);
  }
  __syncthreads();
  T* out = vec + f.vec_off;
  for (int i = tid; i < m; i += NT) out[i] = vl[i];
}

template <typename T>
__global__ __launch_bounds__(NT) void k_sweep_bwd(LevelArgs a, const T* __restrict__ fac,
                                                  T* __restrict__ vec, T* __restrict__ u) {
  extern __shared__ unsigned char smem_raw[];
  T* vl = reinterpret_cast<T*>(smem_raw);
  __shared__ T Ud[DB][DB + 1];
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
  // y - U12 x_q
  for (int r = wv; r < p; r += 4) {
    T d = wave_dot(F + (long long)r * m + p, vl + p, m - p, lane);
    if (lane == 0) vl[r] = csub(vl[r], d);
  }
  __syncthreads();
  // U11 x = y', diagonal blocks from the bottom.
  for (int kb = ((p - 1) / DB) * DB; kb >= 0; kb -= DB) {
    const int nbk = min(DB, p - kb);
    const int c0 = kb + nbk;
    for (int r = kb + wv; r < kb + nbk; r += 4) {
      T d = wave_dot(F + (long long)r * m + c0, vl + c0, p - c0, lane);
      if (lane == 0) vl[r] = csub(vl[r], d);
    }
    for (int t = tid; t < DB * DB; t += NT) {
      int i = t / DB, j = t - i * DB;
      if (i < nbk && j < nbk) Ud[i][j] = F[(long long)(kb + i) * m + kb + j];
    }
    __syncthreads();
    if (wv == 0) {
      T val = lane < nbk ? vl[kb + lane] : czero<T>();
      for (int k = nbk - 1; k >= 0; --k) {
        T xk = (lane == k) ? cdiv(val, Ud[k][k]) : val;
        xk = shfl_c(xk, k);
        if (lane == k) val = xk;
        if (lane < k) val = cfms(Ud[lane][k], xk, val);
      }
      if (lane < nbk) vl[kb + lane] = val;
    }
    __syncthreads();
  }
  const SubDev s = a.subs[f.sub];
  const int* vars = a.vars + f.var_off;
  for (int i = tid; i < m; i += NT) {
    fv[i] = vl[i];
    if (i < p) u[s.u_off + vars[i]] = vl[i];
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
      g_max_lds = v;
    else
      g_max_lds = 65536;
  }
  return g_max_lds;
}

template <typename T, int NB>
void lu_launch(hipStream_t st, const LevelArgs& a, T* fac, int* piv, int* flag, double tau) {
  size_t lds = (size_t)a.max_m * NB * sizeof(T);
  hipLaunchKernelGGL((k_front_lu<T, NB>), dim3(a.nlevel), dim3(NT), lds, st, a, fac, piv, flag, tau);
}

}  // namespace

template <typename T>
void launch_front_assemble(hipStream_t st, const LevelArgs& a, T* fac) {
  hipLaunchKernelGGL(k_front_assemble<T>, dim3(a.nlevel), dim3(NT), 0, st, a, fac);
}

template <typename T>
void launch_front_lu(hipStream_t st, const LevelArgs& a, T* fac, int* piv, int* flag, double tau) {
  // Panel width: as wide as the LDS allows for the largest front of the level.
  size_t budget = (size_t)std::min(max_lds(), 65536) - 1024;
  size_t per_col = (size_t)a.max_m * sizeof(T);
  int nb_max = sizeof(T) == 16 ? 16 : 32;
  int nb = 1;
  while (nb * 2 <= nb_max && per_col * nb * 2 <= budget) nb *= 2;
  if (per_col * nb > budget) throw Error(STF_EINVAL, "front too large for the LDS panel");
  switch (nb) {
    case 32: lu_launch<T, 32>(st, a, fac, piv, flag, tau); break;
    case 16: lu_launch<T, 16>(st, a, fac, piv, flag, tau); break;
    case 8: lu_launch<T, 8>(st, a, fac, piv, flag, tau); break;
    case 4: lu_launch<T, 4>(st, a, fac, piv, flag, tau); break;
    case 2: lu_launch<T, 2>(st, a, fac, piv, flag, tau); break;
    default: lu_launch<T, 1>(st, a, fac, piv, flag, tau); break;
  }
}

template <typename T>
void launch_sweep_fwd(hipStream_t st, const LevelArgs& a, const T* fac, const int* piv, T* vec,
                      const double2* v) {
  size_t lds = (size_t)a.max_m * sizeof(T);
  hipLaunchKernelGGL(k_sweep_fwd<T>, dim3(a.nlevel), dim3(NT), lds, st, a, fac, piv, vec, v);
}

template <typename T>
void launch_sweep_bwd(hipStream_t st, const LevelArgs& a, const T* fac, T* vec, T* u) {
  size_t lds = (size_t)a.max_m * sizeof(T);
  hipLaunchKernelGGL(k_sweep_bwd<T>, dim3(a.nlevel), dim3(NT), lds, st, a, fac, vec, u);
}

template <typename T>
void launch_scatter(hipStream_t st, const T* u, const SubDev* subs, const int4* cover_x,
                    const int4* cover_y, int px, int nx, int ny, double2* z) {
  dim3 blk(64, 4), grd((nx + 63) / 64, (ny + 3) / 4);
  hipLaunchKernelGGL(k_scatter<T>, grd, blk, 0, st, u, subs, cover_x, cover_y, px, nx, ny, z);
}

#define STF_INST(T)                                                                             \
  template void launch_front_assemble<T>(hipStream_t, const LevelArgs&, T*);                    \
  template void launch_front_lu<T>(hipStream_t, const LevelArgs&, T*, int*, int*, double);      \
  template void launch_sweep_fwd<T>(hipStream_t, const LevelArgs&, const T*, const int*, T*,    \
                                    const double2*);                                            \
  template void launch_sweep_bwd<T>(hipStream_t, const LevelArgs&, const T*, T*, T*);           \
  template void launch_scatter<T>(hipStream_t, const T*, const SubDev*, const int4*,            \
                                  const int4*, int, int, int, double2*);
STF_INST(double2)
STF_INST(float2)

}  // namespace stf
