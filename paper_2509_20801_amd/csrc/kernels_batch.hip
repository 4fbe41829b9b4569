// FP64 kernels of the batched flexible GMRES: many independent systems (a
// problem and one of its right-hand sides each) advance in lockstep, every
// kernel covering all of them in one launch.  System s owns the segment
// [off, off + n) of every batch vector (its problem's nx * ny nodes).
//
// Work is cut per system into chunks of CH = 256 * EPT consecutive entries
// (coalesced: entry = base + e * 256 + tid) or, for the stencil, into 64 x 4
// node tiles; a block -> system map gives each block its system, so a launch
// has exactly the blocks the systems need.  Partial sums go to per-block
// slots and are reduced per system over its own block range in a fixed order,
// so every system's arithmetic does not depend on the other systems of the
// batch.
//
// Convergence gating is on the device: act[s] is set at the start of a cycle
// (the FP64 true residual still above tol, iterations left) and cleared by the
// Givens step that meets tol; every per-iteration kernel skips systems with
// act[s] == 0, and the end-of-cycle kernels run for the systems of the cycle
// (cyc[s]).  The host looks at the systems once per cycle.
#include "cplx.h"
#include "stf_internal.h"

namespace stf {

namespace {

constexpr int BT = 256;                      // threads per block (1D kernels)

__device__ inline double bsum256(double v, double* red) {
  v = wave_sum(v);
  const int tid = threadIdx.x + threadIdx.y * blockDim.x;
  __syncthreads();
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

// --- stencil ----------------------------------------------------------------

// y = A x (MODE 0) or y = b - A x with per-tile |y|^2 partials (MODE 1) for
// every system whose gate is set (all systems when gate is null).  Tiles of
// 64 x 4 nodes, 256 threads (64 x 4).
template <int MODE>
__global__ __launch_bounds__(256) void k_bstencil(const double2* __restrict__ x,
                                                  const double2* __restrict__ b,
                                                  double2* __restrict__ y,
                                                  const double2* __restrict__ keps,
                                                  const double2* __restrict__ gc,
                                                  const SysDev* __restrict__ sys,
                                                  const int* __restrict__ tsys,
                                                  const int* __restrict__ gate,
                                                  double* __restrict__ partial) {
  __shared__ double red[4];
  const int t = blockIdx.x;
  const int s = tsys[t];
  if (gate && gate[s] == 0) return;          // whole block
  const SysDev S = sys[s];
  const int lt = t - S.tile0, ntx = (S.nx + 63) / 64;
  const int i = (lt % ntx) * 64 + threadIdx.x;
  const int j = (lt / ntx) * 4 + threadIdx.y;
  const int nx = S.nx, ny = S.ny;
  double loc = 0.0;
  if (i < nx && j < ny) {
    const double2* cxw = gc + S.gc;
    const double2* cxe = cxw + nx;
    const double2* cyw = cxe + nx;
    const double2* cye = cyw + ny;
    const long long n = S.off + (long long)j * nx + i;
    const double2 aw = cxw[i], ae = cxe[i], as = cyw[j], an = cye[j];
    const double2 ke = keps[S.koff + (long long)j * nx + i];
    const double2 dg = make_double2(ke.x - ((aw.x + ae.x) + (as.x + an.x)),
                                    ke.y - ((aw.y + ae.y) + (as.y + an.y)));
    double2 acc = cmul(dg, x[n]);
    if (i > 0) acc = cfma(aw, x[n - 1], acc);
    if (i < nx - 1) acc = cfma(ae, x[n + 1], acc);
    if (j > 0) acc = cfma(as, x[n - nx], acc);
    if (j < ny - 1) acc = cfma(an, x[n + nx], acc);
    if (MODE == 0) {
      y[n] = acc;
    } else {
      const double2 r = csub(b[n], acc);
      y[n] = r;
      loc = r.x * r.x + r.y * r.y;
    }
  }
  if (MODE == 1) {
    const double v = bsum256(loc, red);
    if (threadIdx.x == 0 && threadIdx.y == 0) partial[t] = v;
  }
}

// |v|^2 partials per chunk of 2048 entries (8 per thread).
__global__ __launch_bounds__(BT) void k_bnorm2(const double2* __restrict__ v,
                                               const SysDev* __restrict__ sys,
                                               const int* __restrict__ bsys,
                                               double* __restrict__ npart) {
  __shared__ double red[4];
  const int blk = blockIdx.x, s = bsys[blk];
  const SysDev S = sys[s];
  const long long base = S.off + (long long)(blk - S.blk0[3]) * 2048 + threadIdx.x;
  const long long end = S.off + S.n;
  double a = 0.0;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const long long idx = base + e * BT;
    if (idx < end) {
      const double2 t = v[idx];
      a += t.x * t.x + t.y * t.y;
    }
  }
  const double r = bsum256(a, red);
  if (threadIdx.x == 0) npart[blk] = r;
}

// sc[s * 16 + out] = sum of the system's partials over its tiles (ci < 0) or
// its chunk blocks of size class ci, in a fixed order; gated like the kernel
// that wrote them.
__global__ __launch_bounds__(BT) void k_bsum(const double* __restrict__ partial,
                                             const SysDev* __restrict__ sys, int ci,
                                             const int* __restrict__ gate, double* __restrict__ sc,
                                             int out) {
  __shared__ double red[4];
  const int s = blockIdx.x;
  if (gate && gate[s] == 0) return;
  const SysDev S = sys[s];
  int b0, nb;
  if (ci < 0) {
    b0 = S.tile0;
    nb = ((S.nx + 63) / 64) * ((S.ny + 3) / 4);
  } else {
    b0 = S.blk0[ci];
    nb = S.nblk[ci];
  }
  double a = 0.0;
  for (int b = threadIdx.x; b < nb; b += BT) a += partial[b0 + b];
  const double r = bsum256(a, red);
  if (threadIdx.x == 0) sc[s * 16 + out] = r;
}

// --- Gram-Schmidt -------------------------------------------------------------

// The register-resident Gram-Schmidt passes of the solo solve, per system: a
// thread holds EPT = 32 / NVM entries of each of the nv <= NVM basis vectors
// of its system's chunk.  UPD: w -= V h_s; DOT: partials of V^H w (2 NVM
// reals per block); always the |w|^2 partial.  NRM (with UPD): instead of w,
// v_out = w / |w| with |w|^2 = sc[s][nin] - |h_s|^2 (stored to sc[s][nout] by
// the system's first block).  Skipped for systems with act == 0 and, when
// rgate is given, with rgate == 0.
template <int KT_, int K, int O> __device__ inline void bfold_rec(double* a, int lane) {
  if constexpr (K > 1) {
    const bool up = (lane & O) != 0;
#pragma unroll
    for (int i = 0; i < K / 2; ++i) {
      const double send = up ? a[i] : a[i + K / 2];
      const double keep = up ? a[i + K / 2] : a[i];
      a[i] = keep + __shfl_xor(send, O, 64);
    }
    bfold_rec<KT_, K / 2, O / 2>(a, lane);
  }
}
// Per-wave sums of K values by a folding transpose: lane l ends with the sum
// of value l >> (6 - log2 K) over its lane group.
template <int K> __device__ inline double bwave_fold(double (&a)[K], int lane) {
  static_assert(K >= 2 && K <= 64 && (K & (K - 1)) == 0, "K must be a power of two <= 64");
  bfold_rec<K, K, 32>(a, lane);
  double s = a[0];
#pragma unroll
  for (int o = 32 / K; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  return s;
}

template <int NVM, bool UPD, bool DOT, bool NRM>
__global__ __launch_bounds__(BT) void k_bgs(const double2* __restrict__ V, long long ld, int nv,
                                            const double2* __restrict__ h, int hs,
                                            double2* __restrict__ w,
                                            const SysDev* __restrict__ sys,
                                            const int* __restrict__ bsys, int ci,
                                            const int* __restrict__ act,
                                            const int* __restrict__ rgate,
                                            double* __restrict__ partial,
                                            double* __restrict__ npart,
                                            double2* __restrict__ vout, double* __restrict__ sc,
                                            int nin, int nout) {
  constexpr int K = 2 * NVM;
  constexpr int EPT = 32 / NVM;
  __shared__ double2 hsh[NVM];
  __shared__ double red[4][K];
  __shared__ double nred[4];
  const int blk = blockIdx.x, s = bsys[blk];
  if (act[s] == 0) return;
  if (rgate && rgate[s] == 0) return;
  const SysDev S = sys[s];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int c = blk - S.blk0[ci];
  if (UPD && tid < nv) hsh[tid] = h[(long long)s * hs + tid];
  const long long base = S.off + (long long)c * (BT * EPT) + tid;
  const long long end = S.off + S.n;
  double2 v[NVM][EPT], wr[EPT];
#pragma unroll
  for (int i = 0; i < NVM; ++i)
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const long long idx = base + (long long)e * BT;
      v[i][e] = (idx < end && i < nv) ? V[(long long)i * ld + idx] : make_double2(0.0, 0.0);
    }
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const long long idx = base + (long long)e * BT;
    wr[e] = idx < end ? w[idx] : make_double2(0.0, 0.0);
  }
  if (UPD) {
    __syncthreads();
    double scale = 1.0;
    if (NRM) {
      double hh = 0.0;
      for (int i = 0; i < nv; ++i) hh += hsh[i].x * hsh[i].x + hsh[i].y * hsh[i].y;
      const double n2 = sc[s * 16 + nin] - hh;
      scale = n2 > 0.0 ? 1.0 / sqrt(n2) : 0.0;
      if (c == 0 && tid == 0) sc[s * 16 + nout] = n2 > 0.0 ? n2 : 0.0;
    }
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
#pragma unroll
      for (int i = 0; i < NVM; ++i)
        if (i < nv) wr[e] = cfms(v[i][e], hsh[i], wr[e]);
      const long long idx = base + (long long)e * BT;
      if (idx < end) {
        if (NRM)
          vout[idx] = make_double2(wr[e].x * scale, wr[e].y * scale);
        else
          w[idx] = wr[e];
      }
    }
    if (NRM) return;
  }
  if (DOT) {
    double a[K];
#pragma unroll
    for (int i = 0; i < NVM; ++i) {
      a[2 * i] = fma(v[i][0].y, wr[0].y, v[i][0].x * wr[0].x);         // conj(v) * w
      a[2 * i + 1] = fma(-v[i][0].y, wr[0].x, v[i][0].x * wr[0].y);
#pragma unroll
      for (int e = 1; e < EPT; ++e) {
        a[2 * i] = fma(v[i][e].x, wr[e].x, a[2 * i]);
        a[2 * i] = fma(v[i][e].y, wr[e].y, a[2 * i]);
        a[2 * i + 1] = fma(v[i][e].x, wr[e].y, a[2 * i + 1]);
        a[2 * i + 1] = fma(-v[i][e].y, wr[e].x, a[2 * i + 1]);
      }
    }
    const double sm = bwave_fold<K>(a, lane);
    constexpr int G = 64 / K;
    if ((lane & (G - 1)) == 0) red[wv][lane / G] = sm;
  }
  double nr = 0.0;
#pragma unroll
  for (int e = 0; e < EPT; ++e) nr += wr[e].x * wr[e].x + wr[e].y * wr[e].y;
  nr = wave_sum(nr);
  if (lane == 0) nred[wv] = nr;
  __syncthreads();
  if (DOT && tid < K)
    partial[(long long)blk * K + tid] = (red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]);
  if (tid == 0) npart[blk] = (nred[0] + nred[1]) + (nred[2] + nred[3]);
}

// Between the passes, per system (blockIdx.y): h_s[i] = sum over the system's
// blocks of partial[blk][i] (blocks i < nv), and sc[s][out] = the sum of its
// norm partials (block nv), with ref >= 0 also rgate_out[s] = (out < sc[s][ref] / 2).
// Skipped for systems with act == 0 or, when rgate_in is given, rgate_in == 0.
__global__ __launch_bounds__(BT) void k_bgs_reduce(const double* __restrict__ partial, int K, int nv,
                                                   const SysDev* __restrict__ sys, int ci,
                                                   const int* __restrict__ act,
                                                   const int* __restrict__ rgate_in,
                                                   double2* __restrict__ h, int hs,
                                                   const double* __restrict__ npart,
                                                   double* __restrict__ sc, int out, int ref,
                                                   int* __restrict__ rgate_out) {
  __shared__ double red[4];
  const int i = blockIdx.x, s = blockIdx.y;
  if (act[s] == 0) return;
  if (rgate_in && rgate_in[s] == 0) return;
  const SysDev S = sys[s];
  const int b0 = S.blk0[ci], nb = S.nblk[ci];
  if (i < nv) {
    double sr = 0.0, si = 0.0;
    for (int b = threadIdx.x; b < nb; b += BT) {
      sr += partial[(long long)(b0 + b) * K + 2 * i];
      si += partial[(long long)(b0 + b) * K + 2 * i + 1];
    }
    sr = bsum256(sr, red);
    si = bsum256(si, red);
    if (threadIdx.x == 0) h[(long long)s * hs + i] = make_double2(sr, si);
  } else {
    double a = 0.0;
    for (int b = threadIdx.x; b < nb; b += BT) a += npart[b0 + b];
    a = bsum256(a, red);
    if (threadIdx.x == 0) {
      sc[s * 16 + out] = a;
      if (ref >= 0) rgate_out[s] = (a < 0.5 * sc[s * 16 + ref]) ? 1 : 0;
    }
  }
}

// --- Givens, scaling, cycle control -------------------------------------------

constexpr int BGV = 64;   // largest cycle length of the batched solve (columns staged in LDS)

// The end of Arnoldi step j for every system in one launch.  Blocks < nsys:
// the Givens step of system blockIdx.x (column h1 + h2 when the re-
// orthogonalisation gate is set, with |w|^2 from sc[s][8]), its iteration
// count and history, and the stop decision (estimate <= tol |b|, breakdown, or
// max_iter), which clears act[s].  Other blocks: v_{j+1} = w / |w| on chunks
// of 2048 entries (not needed when the second Gram-Schmidt update wrote it).
// The Givens step writes sc[s][3] only when the gate is set and the scaling
// reads it only when it is not, so the two kinds of blocks do not race.
__global__ __launch_bounds__(BT) void k_bgivens_scale(
    const double2* __restrict__ w, double2* __restrict__ v, const SysDev* __restrict__ sys,
    const int* __restrict__ bsys, int nsys, double2* __restrict__ H, const double2* __restrict__ h1,
    const double2* __restrict__ h2, int m, double* __restrict__ sc, double* __restrict__ cs,
    double2* __restrict__ sn, double2* __restrict__ g, int j, int* __restrict__ act,
    const int* __restrict__ rgate, int* __restrict__ kcol, int* __restrict__ it,
    double* __restrict__ hist, int hcap, double tol, int max_iter) {
  __shared__ double2 col[BGV + 1];
  __shared__ double scs[BGV];
  __shared__ double2 ssn[BGV];
  if ((int)blockIdx.x >= nsys) {
    const int blk = blockIdx.x - nsys, s = bsys[blk];
    if (act[s] == 0 || rgate[s] != 0) return;
    const SysDev S = sys[s];
    const double s2 = sc[s * 16 + 3];
    const double inv = s2 > 0.0 ? 1.0 / sqrt(s2) : 0.0;
    const long long base = S.off + (long long)(blk - S.blk0[3]) * 2048 + threadIdx.x;
    const long long end = S.off + S.n;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const long long idx = base + e * BT;
      if (idx < end) {
        const double2 a = w[idx];
        v[idx] = make_double2(a.x * inv, a.y * inv);
      }
    }
    return;
  }
  const int s = blockIdx.x, t = threadIdx.x;
  if (act[s] == 0) return;
  const bool second = rgate[s] != 0;
  const int hs = m + 1;
  double* q = sc + s * 16;
  double* css = cs + (long long)s * m;
  double2* sns = sn + (long long)s * m;
  double2* gs = g + (long long)s * hs;
  for (int i = t; i <= j; i += BT) {
    const double2 a = h1[(long long)s * hs + i];
    col[i] = second ? cadd(a, h2[(long long)s * hs + i]) : a;
  }
  for (int i = t; i < j; i += BT) {
    scs[i] = css[i];
    ssn[i] = sns[i];
  }
  __syncthreads();
  if (t == 0) {
    const double n2 = second ? q[8] : q[3];
    if (second) q[3] = n2;
    col[j + 1] = make_double2(sqrt(n2), 0.0);
    for (int i = 0; i < j; ++i) {
      const double c = scs[i];
      const double2 sv = ssn[i];
      const double2 a = col[i], b = col[i + 1];
      // [c, s; -conj(s), c] [a; b]
      col[i] = make_double2(c * a.x + (sv.x * b.x - sv.y * b.y), c * a.y + (sv.x * b.y + sv.y * b.x));
      col[i + 1] = make_double2(-(sv.x * a.x + sv.y * a.y) + c * b.x, -(sv.x * a.y - sv.y * a.x) + c * b.y);
    }
    const double2 a = col[j], b = col[j + 1];
    const double na = hypot(a.x, a.y), nb = hypot(b.x, b.y);
    double c;
    double2 sv, r;
    if (nb == 0.0) {
      c = 1.0; sv = make_double2(0.0, 0.0); r = a;
    } else if (na == 0.0) {
      c = 0.0; sv = make_double2(b.x / nb, -b.y / nb); r = make_double2(nb, 0.0);
    } else {
      const double nrm = hypot(na, nb);
      const double2 ph = make_double2(a.x / na, a.y / na);
      c = na / nrm;
      sv = make_double2((ph.x * b.x + ph.y * b.y) / nrm, (ph.y * b.x - ph.x * b.y) / nrm);
      r = make_double2(ph.x * nrm, ph.y * nrm);
    }
    css[j] = c;
    sns[j] = sv;
    col[j] = r;
    col[j + 1] = make_double2(0.0, 0.0);
    const double2 gj = gs[j];
    const double2 g1 = make_double2(-(sv.x * gj.x + sv.y * gj.y), -(sv.x * gj.y - sv.y * gj.x));
    gs[j + 1] = g1;
    gs[j] = make_double2(c * gj.x, c * gj.y);
    const double est = hypot(g1.x, g1.y);
    q[4] = est;
    const int k = it[s] + 1;
    it[s] = k;
    kcol[s] = j + 1;
    const double bn = sqrt(q[0]);
    if (k < hcap) hist[(long long)s * hcap + k] = est / bn;
    if (!isfinite(est)) q[10] = 1.0;
    if (!(est > tol * bn) || n2 == 0.0 || k >= max_iter) act[s] = 0;
  }
  __syncthreads();
  double2* Hc = H + (long long)s * hs * m + (long long)j * hs;
  for (int i = t; i <= j + 1; i += BT) Hc[i] = col[i];
}

// pact[p] = 1 while a right-hand side of problem p is active (systems are
// slot-major: s = slot * nprob + p).
__global__ __launch_bounds__(BT) void k_bpact(const int* __restrict__ act, int nslot, int nprob,
                                              int* __restrict__ pact) {
  for (int p = threadIdx.x; p < nprob; p += BT) {
    int a = 0;
    for (int k = 0; k < nslot; ++k) a |= act[k * nprob + p];
    pact[p] = a;
  }
}

// Start of a cycle.  Blocks < nsys: system blockIdx.x joins the cycle (act =
// cyc = 1) when it is present, |b| > 0, its FP64 true residual sc[s][2] is
// above tol |b| and finite, and iterations are left; g = (|r|, 0, ...);
// kcol = 0.  Other blocks: v_0 = r / |r| on chunks of 2048 entries (for every
// system with |r| > 0; it does not depend on the decision).
__global__ __launch_bounds__(BT) void k_bcycle_start(
    const double2* __restrict__ r, double2* __restrict__ v, const SysDev* __restrict__ sys,
    const int* __restrict__ bsys, int nsys, const double* __restrict__ sc, double2* __restrict__ g,
    int glen, int* __restrict__ act, int* __restrict__ cyc, int* __restrict__ kcol,
    const int* __restrict__ it, double tol, int max_iter) {
  if ((int)blockIdx.x >= nsys) {
    const int blk = blockIdx.x - nsys, s = bsys[blk];
    const SysDev S = sys[s];
    const double s2 = sc[s * 16 + 2];
    if (!(s2 > 0.0)) return;
    const double inv = 1.0 / sqrt(s2);
    const long long base = S.off + (long long)(blk - S.blk0[3]) * 2048 + threadIdx.x;
    const long long end = S.off + S.n;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const long long idx = base + e * BT;
      if (idx < end) {
        const double2 a = r[idx];
        v[idx] = make_double2(a.x * inv, a.y * inv);
      }
    }
    return;
  }
  const int s = blockIdx.x;
  const double b2 = sc[s * 16 + 0], r2 = sc[s * 16 + 2];
  const double bn = sqrt(b2), rn = sqrt(r2);
  for (int i = threadIdx.x; i < glen; i += BT)
    g[(long long)s * glen + i] = make_double2(i == 0 ? rn : 0.0, 0.0);
  if (threadIdx.x == 0) {
    const int on = sys[s].present && b2 > 0.0 && isfinite(r2) && rn > tol * bn && it[s] < max_iter;
    act[s] = on;
    cyc[s] = on;
    kcol[s] = 0;
  }
}

// y_s = R_s^{-1} g_s (kcol[s] columns) for the systems of the cycle, one block
// each, thread 0 substituting from LDS.
__global__ void k_btrisolve(const double2* __restrict__ H, int m, const double2* __restrict__ g,
                            double2* __restrict__ y, const int* __restrict__ kcol,
                            const int* __restrict__ cyc) {
  __shared__ double2 R[BGV * BGV];
  __shared__ double2 gsh[BGV], ys[BGV];
  const int s = blockIdx.x;
  const int k = kcol[s];
  if (cyc[s] == 0 || k == 0) return;
  const int hs = m + 1;
  const double2* Hs = H + (long long)s * hs * m;
  for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
    const int c = e / k, r = e - c * k;
    if (r <= c) R[c * BGV + r] = Hs[(long long)c * hs + r];
  }
  for (int i = threadIdx.x; i < k; i += blockDim.x) gsh[i] = g[(long long)s * hs + i];
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int i = k - 1; i >= 0; --i) {
    double2 a = gsh[i];
    for (int t = i + 1; t < k; ++t) a = cfms(R[t * BGV + i], ys[t], a);
    ys[i] = cdiv(a, R[i * BGV + i]);
    y[(long long)s * hs + i] = ys[i];
  }
}

// x += Z_s y_s over kcol[s] vectors, chunks of 2048 entries.
__global__ __launch_bounds__(BT) void k_bxupdate(const double2* __restrict__ Z, long long ld,
                                                 const double2* __restrict__ y, int hs,
                                                 double2* __restrict__ x,
                                                 const SysDev* __restrict__ sys,
                                                 const int* __restrict__ bsys,
                                                 const int* __restrict__ kcol,
                                                 const int* __restrict__ cyc) {
  __shared__ double2 ysh[BGV];
  const int blk = blockIdx.x, s = bsys[blk];
  const int k = kcol[s];
  if (cyc[s] == 0 || k == 0) return;
  if ((int)threadIdx.x < k) ysh[threadIdx.x] = y[(long long)s * hs + threadIdx.x];
  __syncthreads();
  const SysDev S = sys[s];
  const long long base = S.off + (long long)(blk - S.blk0[3]) * 2048 + threadIdx.x;
  const long long end = S.off + S.n;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const long long idx = base + e * BT;
    if (idx < end) {
      double2 a = x[idx];
      for (int i = 0; i < k; ++i) a = cfma(Z[(long long)i * ld + idx], ysh[i], a);
      x[idx] = a;
    }
  }
}

// Per system, to device-visible host memory: |r|^2, iterations, cycle flag,
// non-finite flag (4 doubles each).
__global__ __launch_bounds__(BT) void k_bstatus(const double* __restrict__ sc,
                                                const int* __restrict__ it,
                                                const int* __restrict__ cyc, int nsys,
                                                double* __restrict__ out) {
  for (int s = threadIdx.x; s < nsys; s += BT) {
    out[4 * s + 0] = sc[s * 16 + 2];
    out[4 * s + 1] = (double)it[s];
    out[4 * s + 2] = (double)cyc[s];
    out[4 * s + 3] = sc[s * 16 + 10];
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

void launch_bstencil(hipStream_t st, int mode, const double2* x, const double2* b, double2* y,
                     const double2* keps, const double2* gc, const SysDev* sys, const int* tsys,
                     int ntiles, const int* gate, double* partial) {
  if (ntiles <= 0) return;
  const dim3 blk(64, 4);
  if (mode == 0)
    STF_LAUNCH(k_bstencil<0>, dim3(ntiles), blk, 0, st, x, b, y, keps, gc, sys, tsys, gate,
                       partial);
  else
    STF_LAUNCH(k_bstencil<1>, dim3(ntiles), blk, 0, st, x, b, y, keps, gc, sys, tsys, gate,
                       partial);
}

void launch_bnorm2(hipStream_t st, const double2* v, const SysDev* sys, const int* bsys, int nblk,
                   double* npart) {
  if (nblk > 0) STF_LAUNCH(k_bnorm2, dim3(nblk), dim3(BT), 0, st, v, sys, bsys, npart);
}

void launch_bsum(hipStream_t st, const double* partial, const SysDev* sys, int nsys, int ci,
                 const int* gate, double* sc, int out) {
  STF_LAUNCH(k_bsum, dim3(nsys), dim3(BT), 0, st, partial, sys, ci, gate, sc, out);
}

int bgs_class(int nv) { return nv <= 8 ? 2 : nv <= 16 ? 1 : nv <= 32 ? 0 : -1; }

void launch_bgs(hipStream_t st, int mode, const double2* V, long long ld, int nv, const double2* h,
                int hs, double2* w, const SysDev* sys, const int* bsys, int nblk, const int* act,
                const int* rgate, double* partial, double* npart, double2* vout, double* sc, int nin,
                int nout) {
  const int ci = bgs_class(nv);
  STF_REQUIRE(ci >= 0 && nv >= 1, "batched Gram-Schmidt takes 1..32 basis vectors");
  if (nblk <= 0) return;
  const dim3 g(nblk), b(BT);
#define STF_BGS_CASE(M)                                                                          \
  if (M == (32 >> ci)) {                                                                         \
    if (mode == GS_DOT)                                                                          \
      STF_LAUNCH((k_bgs<M, false, true, false>), g, b, 0, st, V, ld, nv, h, hs, w, sys,  \
                         bsys, ci, act, rgate, partial, npart, vout, sc, nin, nout);             \
    else if (mode == GS_UPDATE_DOT)                                                              \
      STF_LAUNCH((k_bgs<M, true, true, false>), g, b, 0, st, V, ld, nv, h, hs, w, sys,   \
                         bsys, ci, act, rgate, partial, npart, vout, sc, nin, nout);             \
    else                                                                                         \
      STF_LAUNCH((k_bgs<M, true, false, true>), g, b, 0, st, V, ld, nv, h, hs, w, sys,   \
                         bsys, ci, act, rgate, partial, npart, vout, sc, nin, nout);             \
    return;                                                                                      \
  }
  STF_BGS_CASE(8)
  STF_BGS_CASE(16)
  STF_BGS_CASE(32)
#undef STF_BGS_CASE
}

void launch_bgs_reduce(hipStream_t st, const double* partial, int nv, const SysDev* sys, int nsys,
                       const int* act, const int* rgate_in, double2* h, int hs, const double* npart,
                       double* sc, int out, int ref, int* rgate_out) {
  const int ci = bgs_class(nv);
  const int K = 2 * (ci == 2 ? 8 : ci == 1 ? 16 : 32);
  STF_LAUNCH(k_bgs_reduce, dim3(nv + 1, nsys), dim3(BT), 0, st, partial, K, nv, sys, ci, act,
                     rgate_in, h, hs, npart, sc, out, ref, rgate_out);
}

void launch_bgivens_scale(hipStream_t st, const double2* w, double2* v, const SysDev* sys,
                          const int* bsys, int nblk, int nsys, double2* H, const double2* h1,
                          const double2* h2, int m, double* sc, double* cs, double2* sn, double2* g,
                          int j, int* act, const int* rgate, int* kcol, int* it, double* hist,
                          int hcap, double tol, int max_iter) {
  STF_REQUIRE(m <= BGV && j < m, "batched Givens step beyond the staged column");
  STF_LAUNCH(k_bgivens_scale, dim3(nsys + nblk), dim3(BT), 0, st, w, v, sys, bsys, nsys, H,
                     h1, h2, m, sc, cs, sn, g, j, act, rgate, kcol, it, hist, hcap, tol, max_iter);
}

void launch_bpact(hipStream_t st, const int* act, int nslot, int nprob, int* pact) {
  STF_LAUNCH(k_bpact, dim3(1), dim3(BT), 0, st, act, nslot, nprob, pact);
}

void launch_bcycle_start(hipStream_t st, const double2* r, double2* v, const SysDev* sys,
                         const int* bsys, int nblk, int nsys, const double* sc, double2* g, int glen,
                         int* act, int* cyc, int* kcol, const int* it, double tol, int max_iter) {
  STF_LAUNCH(k_bcycle_start, dim3(nsys + nblk), dim3(BT), 0, st, r, v, sys, bsys, nsys, sc, g,
                     glen, act, cyc, kcol, it, tol, max_iter);
}

void launch_btrisolve(hipStream_t st, const double2* H, int m, const double2* g, double2* y,
                      const int* kcol, const int* cyc, int nsys) {
  STF_REQUIRE(m <= BGV, "batched triangular solve beyond the staged size");
  STF_LAUNCH(k_btrisolve, dim3(nsys), dim3(64), 0, st, H, m, g, y, kcol, cyc);
}

void launch_bxupdate(hipStream_t st, const double2* Z, long long ld, const double2* y, int hs,
                     double2* x, const SysDev* sys, const int* bsys, int nblk, const int* kcol,
                     const int* cyc) {
  if (nblk > 0)
    STF_LAUNCH(k_bxupdate, dim3(nblk), dim3(BT), 0, st, Z, ld, y, hs, x, sys, bsys, kcol, cyc);
}

void launch_bstatus(hipStream_t st, const double* sc, const int* it, const int* cyc, int nsys,
                    double* host_out) {
  STF_LAUNCH(k_bstatus, dim3(1), dim3(BT), 0, st, sc, it, cyc, nsys, host_out);
}

}  // namespace stf
