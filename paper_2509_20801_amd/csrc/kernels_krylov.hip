// FP64 kernels of the flexible GMRES outer iteration: classical Gram-Schmidt
// with selective re-orthogonalisation (a block dot pass that also yields |w|^2,
// a block update pass that yields the new |w|^2, and a second pass only when
// the norm dropped below |w|/sqrt(2), decided on the device), complex Givens
// rotations and the solution update x += Z y.
//
// Vectors are contiguous complex128 arrays of n entries; a basis V stores its
// vectors with leading dimension ld.  Every thread owns up to EPT entries of a
// chunk of EPT*256 consecutive entries (coalesced: entry = base + e*256 + tid),
// keeps w in registers and walks the basis; partial sums per workgroup go to
// a buffer reduced by a second kernel in a fixed order, so results do not
// depend on scheduling.
#include "cplx.h"
#include "stf_internal.h"

namespace stf {

namespace {

constexpr int KT = 256;
constexpr int EPT = 8;
constexpr int CHUNK = KT * EPT;
constexpr int VB = 4;    // basis vectors per pass of the dot kernel

__device__ inline double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int tid = threadIdx.x;
  __syncthreads();
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

// partial[blk][i] = V_i^H w over the block's chunk; with `gate`, skipped
// (all threads return) unless *gate != 0; with `norm_partial`, also |w|^2.
__global__ __launch_bounds__(KT) void k_mdot(const double2* __restrict__ V, long long ld, int nv,
                                             const double2* __restrict__ w, long long n,
                                             double2* __restrict__ partial,
                                             double* __restrict__ norm_partial,
                                             const int* __restrict__ gate) {
  __shared__ double red[4];
  if (gate && gate[0] == 0) return;
  const long long base = (long long)blockIdx.x * CHUNK + threadIdx.x;
  double2 wr[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    long long idx = base + (long long)e * KT;
    wr[e] = idx < n ? w[idx] : make_double2(0.0, 0.0);
  }
  for (int i0 = 0; i0 < nv; i0 += VB) {
    double2 acc[VB];
#pragma unroll
    for (int b = 0; b < VB; ++b) acc[b] = make_double2(0.0, 0.0);
#pragma unroll
    for (int b = 0; b < VB; ++b) {
      if (i0 + b < nv) {
        const double2* vi = V + (long long)(i0 + b) * ld;
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
          long long idx = base + (long long)e * KT;
          if (idx < n) {
            double2 a = vi[idx];
            // conj(a) * w
            acc[b].x = fma(a.x, wr[e].x, acc[b].x);
            acc[b].x = fma(a.y, wr[e].y, acc[b].x);
            acc[b].y = fma(a.x, wr[e].y, acc[b].y);
            acc[b].y = fma(-a.y, wr[e].x, acc[b].y);
          }
        }
      }
    }
#pragma unroll
    for (int b = 0; b < VB; ++b) {
      double sr = block_sum(acc[b].x, red);
      double si = block_sum(acc[b].y, red);
      if (threadIdx.x == 0 && i0 + b < nv)
        partial[(long long)blockIdx.x * nv + i0 + b] = make_double2(sr, si);
    }
  }
  if (norm_partial) {
    double nr = 0.0;
#pragma unroll
    for (int e = 0; e < EPT; ++e) nr += wr[e].x * wr[e].x + wr[e].y * wr[e].y;
    double t = block_sum(nr, red);
    if (threadIdx.x == 0) norm_partial[blockIdx.x] = t;
  }
}

// h[i] = sum_b partial[b * stride + i] in a fixed order (skipped unless *gate when gated).
__global__ __launch_bounds__(KT) void k_mdot_reduce(const double2* __restrict__ partial, int nblk,
                                                    int stride, double2* __restrict__ h,
                                                    const int* __restrict__ gate) {
  __shared__ double red[4];
  if (gate && gate[0] == 0) return;
  const int i = blockIdx.x;
  double sr = 0.0, si = 0.0;
  for (int b = threadIdx.x; b < nblk; b += KT) {
    double2 v = partial[(long long)b * stride + i];
    sr += v.x;
    si += v.y;
  }
  sr = block_sum(sr, red);
  si = block_sum(si, red);
  if (threadIdx.x == 0) h[i] = make_double2(sr, si);
}

// w -= V h; optional per-block |w|^2 partials.
__global__ __launch_bounds__(KT) void k_mupdate(const double2* __restrict__ V, long long ld, int nv,
                                                const double2* __restrict__ h,
                                                double2* __restrict__ w, long long n,
                                                double* __restrict__ norm_partial,
                                                const int* __restrict__ gate) {
  __shared__ double red[4];
  __shared__ double2 hs[256];
  if (gate && gate[0] == 0) return;
  const long long base = (long long)blockIdx.x * CHUNK + threadIdx.x;
  double2 wr[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    long long idx = base + (long long)e * KT;
    wr[e] = idx < n ? w[idx] : make_double2(0.0, 0.0);
  }
  for (int i0 = 0; i0 < nv; i0 += 256) {
    int cnt = nv - i0 < 256 ? nv - i0 : 256;
    __syncthreads();
    if ((int)threadIdx.x < cnt) hs[threadIdx.x] = h[i0 + threadIdx.x];
    __syncthreads();
    for (int b = 0; b < cnt; ++b) {
      const double2* vi = V + (long long)(i0 + b) * ld;
      const double2 hb = hs[b];
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        long long idx = base + (long long)e * KT;
        if (idx < n) wr[e] = cfms(vi[idx], hb, wr[e]);
      }
    }
  }
  double nr = 0.0;
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    long long idx = base + (long long)e * KT;
    if (idx < n) {
      w[idx] = wr[e];
      nr += wr[e].x * wr[e].x + wr[e].y * wr[e].y;
    }
  }
  if (norm_partial) {
    double s = block_sum(nr, red);
    if (threadIdx.x == 0) norm_partial[blockIdx.x] = s;
  }
}

// Register-resident Gram-Schmidt passes for bases of at most 32 vectors: each
// thread holds 32 basis values in registers, EPT = 32 / NVM entries of each of
// the NVM vectors (coalesced: entry = base + e * 256 + tid), all loaded at once.  UPD: w -= V h; DOT: the
// partial products V^H w of the (updated) entries, written as
// partial[blk][NVM] (complex); always the partial |w|^2.  With UPD and DOT
// together one read of the basis serves the update of the first pass and the
// products of the second.
//
// The per-wave sums of the 2*NVM real values use a folding transpose: at each
// exchange a lane keeps one half of its values and adds the partner's other
// half, so after log2(2*NVM) exchanges lane l holds the sum of value
// l >> (6 - log2(2*NVM)) over its lane group (63 exchanges for 64 values
// instead of 384 for separate butterflies).
// One exchange of the fold on the first K values (offset O), then the next.
// Recursion on compile-time K keeps every index constant, so the values stay
// in registers.
template <int KT_, int K, int O> __device__ inline void fold_rec(double* a, int lane) {
  if constexpr (K > 1) {
    const bool up = (lane & O) != 0;
#pragma unroll
    for (int i = 0; i < K / 2; ++i) {
      const double send = up ? a[i] : a[i + K / 2];
      const double keep = up ? a[i + K / 2] : a[i];
      a[i] = keep + __shfl_xor(send, O, 64);
    }
    fold_rec<KT_, K / 2, O / 2>(a, lane);
  }
}
template <int K> __device__ inline double wave_fold(double (&a)[K], int lane) {
  static_assert(K >= 2 && K <= 64 && (K & (K - 1)) == 0, "K must be a power of two <= 64");
  fold_rec<K, K, 32>(a, lane);
  double s = a[0];
#pragma unroll
  for (int o = 32 / K; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  return s;
}

// NRM (with UPD, without DOT): the update of a second pass whose result is
// final; instead of w it writes v = w / |w| to vout, with |w|^2 taken as
// nrm_in[0] - |h|^2 (the new w is orthogonal to the basis, so the norm removed
// is that of the coefficients), which block 0 also stores in nrm_out[0].
// One launch serves the right-hand sides of a GsSet: blockIdx.y selects the
// pointers, the pass over each vector is that of a single launch.
template <int NVM, bool UPD, bool DOT, bool NRM>
__global__ __launch_bounds__(KT) void k_gs(GsSet S, long long ld, int nv, long long n) {
  const int sy = blockIdx.y;
  const double2* __restrict__ V = S.V[sy];
  const double2* __restrict__ h = S.h[sy];
  double2* __restrict__ w = S.w[sy];
  double* __restrict__ partial = reinterpret_cast<double*>(S.partial[sy]);
  double* __restrict__ norm_partial = S.npart[sy];
  const int* __restrict__ gate = S.gate[sy];
  double2* __restrict__ vout = S.vout[sy];
  const double* __restrict__ nrm_in = S.nrm_in[sy];
  double* __restrict__ nrm_out = S.nrm_out[sy];
  constexpr int K = 2 * NVM;
  constexpr int EPT = 32 / NVM;                          // entries per thread
  __shared__ double2 hs[NVM];
  __shared__ double red[4][K];
  __shared__ double nred[4];
  if (gate && gate[0] == 0) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (UPD && tid < nv) hs[tid] = h[tid];
  const long long base = (long long)blockIdx.x * (KT * EPT) + tid;
  double2 v[NVM][EPT], wr[EPT];
#pragma unroll
  for (int i = 0; i < NVM; ++i)
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const long long idx = base + (long long)e * KT;
      v[i][e] = (idx < n && i < nv) ? V[(long long)i * ld + idx] : make_double2(0.0, 0.0);
    }
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const long long idx = base + (long long)e * KT;
    wr[e] = idx < n ? w[idx] : make_double2(0.0, 0.0);
  }
  if (UPD) {
    __syncthreads();
    double scale = 1.0;
    if (NRM) {
      double hh = 0.0;
      for (int i = 0; i < nv; ++i) hh += hs[i].x * hs[i].x + hs[i].y * hs[i].y;
      const double n2 = nrm_in[0] - hh;
      scale = n2 > 0.0 ? 1.0 / sqrt(n2) : 0.0;
      if (blockIdx.x == 0 && tid == 0) nrm_out[0] = n2 > 0.0 ? n2 : 0.0;
    }
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
#pragma unroll
      for (int i = 0; i < NVM; ++i)
        if (i < nv) wr[e] = cfms(v[i][e], hs[i], wr[e]);
      const long long idx = base + (long long)e * KT;
      if (idx < n) {
        if (NRM)
          vout[idx] = make_double2(wr[e].x * scale, wr[e].y * scale);
        else
          w[idx] = wr[e];
      }
    }
    if (NRM) return;                         // no partials needed
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
    const double s = wave_fold<K>(a, lane);
    constexpr int G = 64 / K;                              // lanes per value
    if ((lane & (G - 1)) == 0) red[wv][lane / G] = s;
  }
  double nr = 0.0;
#pragma unroll
  for (int e = 0; e < EPT; ++e) nr += wr[e].x * wr[e].x + wr[e].y * wr[e].y;
  nr = wave_sum(nr);
  if (lane == 0) nred[wv] = nr;
  __syncthreads();
  if (DOT && tid < K)
    partial[(long long)blockIdx.x * K + tid] = (red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]);
  if (tid == 0) norm_partial[blockIdx.x] = (nred[0] + nred[1]) + (nred[2] + nred[3]);
}

// Fixed-order sum of n partials into out[0].  With `decide`: out holds the
// new |w|^2 and ref[0] the |w|^2 before the update; gate[0] is set to 1 when
// the update cancelled more than half of the norm squared (re-orthogonalise),
// else 0.  With `gate` alone the kernel runs only when gate[0] != 0.
__global__ __launch_bounds__(KT) void k_norm_reduce(const double* __restrict__ partial, int n,
                                                    double* __restrict__ out,
                                                    const double* __restrict__ ref,
                                                    int* __restrict__ gate, int decide) {
  __shared__ double red[4];
  if (!decide && gate && gate[0] == 0) return;
  double s = 0.0;
  for (int t = threadIdx.x; t < n; t += KT) s += partial[t];
  s = block_sum(s, red);
  if (threadIdx.x == 0) {
    out[0] = s;
    if (decide) gate[0] = (s < 0.5 * ref[0]) ? 1 : 0;
  }
}

// sum_{b = t, t + KT, ... < n} x[b * stride] in that order, the loads issued
// eight at a time (one memory round trip per eight terms).
template <typename V, typename F>
__device__ inline void strided_sum(int t, int n, F load, V& acc) {
  constexpr int LB = 8;
  for (int b0 = t; b0 < n; b0 += LB * KT) {
    V v[LB];
#pragma unroll
    for (int u = 0; u < LB; ++u) {
      const int b = b0 + u * KT;
      v[u] = b < n ? load(b) : V{};
    }
#pragma unroll
    for (int u = 0; u < LB; ++u) acc += v[u];
  }
}
struct Cd {
  double x = 0.0, y = 0.0;
  __device__ Cd& operator+=(const Cd& o) {
    x += o.x;
    y += o.y;
    return *this;
  }
};

// The reductions between the register Gram-Schmidt passes, one launch each.
// Blocks 0..nv-1: h[i] = sum_b partial[b * stride + i] in a fixed order;
// block nv: out[0] = sum of the nblk norm partials and, with ref, the
// re-orthogonalisation gate (out < ref/2).
__global__ __launch_bounds__(KT) void k_gs_reduce(GsRedSet S, int nblk, int stride, int nv) {
  const int sy = blockIdx.y;
  const double2* __restrict__ partial = S.partial[sy];
  double2* __restrict__ h = S.h[sy];
  const double* __restrict__ npart = S.npart[sy];
  double* __restrict__ out = S.out[sy];
  const double* __restrict__ ref = S.ref[sy];
  int* __restrict__ gate = S.gate[sy];
  __shared__ double red[4];
  const int i = blockIdx.x;
  if (i < nv) {
    Cd acc;
    strided_sum(threadIdx.x, nblk, [&](int b) {
      const double2 v = partial[(long long)b * stride + i];
      Cd c;
      c.x = v.x;
      c.y = v.y;
      return c;
    }, acc);
    const double sr = block_sum(acc.x, red);
    const double si = block_sum(acc.y, red);
    if (threadIdx.x == 0) h[i] = make_double2(sr, si);
  } else {
    double s = 0.0;
    strided_sum(threadIdx.x, nblk, [&](int b) { return npart[b]; }, s);
    s = block_sum(s, red);
    if (threadIdx.x == 0) {
      out[0] = s;
      if (ref) gate[0] = (s < 0.5 * ref[0]) ? 1 : 0;
    }
  }
}

// h1 += h2 when gate[0] != 0 (accumulates the re-orthogonalisation coefficients).
__global__ void k_hacc(double2* __restrict__ h1, const double2* __restrict__ h2, int nv,
                       const int* __restrict__ gate) {
  if (gate[0] == 0) return;
  for (int i = threadIdx.x; i < nv; i += blockDim.x)
    h1[i] = make_double2(h1[i].x + h2[i].x, h1[i].y + h2[i].y);
}

__device__ inline void scale_body(const double2* __restrict__ w, const double* __restrict__ nrm2,
                                  double2* __restrict__ v, long long n, const int* __restrict__ skip,
                                  int blk, int nblk) {
  if (skip && skip[0] != 0) return;
  const double s2 = nrm2[0];
  const double inv = s2 > 0.0 ? 1.0 / sqrt(s2) : 0.0;
  for (long long t = (long long)blk * KT + threadIdx.x; t < n; t += (long long)nblk * KT) {
    double2 a = w[t];
    v[t] = make_double2(a.x * inv, a.y * inv);
  }
}

__global__ __launch_bounds__(KT) void k_scale(const double2* __restrict__ w,
                                              const double* __restrict__ nrm2,
                                              double2* __restrict__ v, long long n,
                                              const int* __restrict__ skip) {
  scale_body(w, nrm2, v, n, skip, blockIdx.x, gridDim.x);
}

// The start of an FGMRES cycle: v_0 = r / |r| (|r|^2 in nrm2[0]), and block 0
// also sets g = (|r|, 0, ..., 0) (glen entries), all from device values.
__global__ __launch_bounds__(KT) void k_cycle_start(CycleSet S, long long n, int glen) {
  const int sy = blockIdx.y;
  const double2* __restrict__ r = S.r[sy];
  const double* __restrict__ nrm2 = S.nrm2[sy];
  double2* __restrict__ v = S.v[sy];
  double2* __restrict__ g = S.gs[sy];
  if (blockIdx.x == 0)
    for (int i = threadIdx.x; i < glen; i += KT)
      g[i] = make_double2(i == 0 ? sqrt(nrm2[0]) : 0.0, 0.0);
  scale_body(r, nrm2, v, n, nullptr, blockIdx.x, gridDim.x);
}

// One Givens step of FGMRES for column j.
//   column j of the Hessenberg matrix: h[i] (i <= j), h[j+1] = |w|.
//   Earlier rotations are applied, a new one zeroes h[j+1], g is rotated and
//   est = |g[j+1]| is the residual norm of the least-squares iterate.
// The operands are staged in LDS by the whole block (j < GV), so that the
// sequential rotations by thread 0 wait on no memory round trips.
constexpr int GV = 256;
// With gate (and gate[0] != 0): the column is h + h2 and |w|^2 is wnorm2_alt[0],
// which is also stored to wnorm2[0].
__device__ inline void givens_body(double2* __restrict__ H, const double2* __restrict__ h,
                                               double* __restrict__ wnorm2,
                                               double* __restrict__ cs, double2* __restrict__ sn,
                                               double2* __restrict__ g, int j, int ldh,
                                               double* __restrict__ est,
                                               const double2* __restrict__ h2,
                                               const int* __restrict__ gate,
                                               const double* __restrict__ wnorm2_alt,
                                               double* __restrict__ host_out) {
  __shared__ double2 col[GV + 1];
  __shared__ double scs[GV];
  __shared__ double2 ssn[GV];
  const int t = threadIdx.x;
  const bool second = gate && gate[0] != 0;
  for (int i = t; i <= j; i += blockDim.x)
    col[i] = second ? make_double2(h[i].x + h2[i].x, h[i].y + h2[i].y) : h[i];
  for (int i = t; i < j; i += blockDim.x) {
    scs[i] = cs[i];
    ssn[i] = sn[i];
  }
  if (t == 0) {
    const double n2 = second ? wnorm2_alt[0] : wnorm2[0];
    if (second) wnorm2[0] = n2;
    col[j + 1] = make_double2(sqrt(n2), 0.0);
  }
  __syncthreads();
  if (t == 0) {
    for (int i = 0; i < j; ++i) {
      const double c = scs[i];
      const double2 s = ssn[i];
      const double2 a = col[i], b = col[i + 1];
      // [c, s; -conj(s), c] [a; b]
      col[i] = make_double2(c * a.x + (s.x * b.x - s.y * b.y), c * a.y + (s.x * b.y + s.y * b.x));
      col[i + 1] = make_double2(-(s.x * a.x + s.y * a.y) + c * b.x, -(s.x * a.y - s.y * a.x) + c * b.y);
    }
    const double2 a = col[j], b = col[j + 1];
    const double na = hypot(a.x, a.y), nb = hypot(b.x, b.y);
    double c;
    double2 s, r;
    if (nb == 0.0) {
      c = 1.0; s = make_double2(0.0, 0.0); r = a;
    } else if (na == 0.0) {
      c = 0.0; s = make_double2(b.x / nb, -b.y / nb); r = make_double2(nb, 0.0);
    } else {
      const double nrm = hypot(na, nb);
      const double2 ph = make_double2(a.x / na, a.y / na);          // a / |a|
      c = na / nrm;
      // s = (a/|a|) conj(b) / nrm
      s = make_double2((ph.x * b.x + ph.y * b.y) / nrm, (ph.y * b.x - ph.x * b.y) / nrm);
      r = make_double2(ph.x * nrm, ph.y * nrm);
    }
    cs[j] = c;
    sn[j] = s;
    col[j] = r;
    col[j + 1] = make_double2(0.0, 0.0);
    const double2 gj = g[j];
    // g[j+1] = -conj(s) g[j]; g[j] = c g[j]
    const double2 g1 = make_double2(-(s.x * gj.x + s.y * gj.y), -(s.x * gj.y - s.y * gj.x));
    g[j + 1] = g1;
    g[j] = make_double2(c * gj.x, c * gj.y);
    est[0] = hypot(g1.x, g1.y);
    if (host_out) {                          // |w|^2 and the estimate, straight to the host
      host_out[0] = second ? wnorm2_alt[0] : wnorm2[0];
      host_out[1] = est[0];
    }
  }
  __syncthreads();
  double2* Hc = H + (long long)j * ldh;
  for (int i = t; i <= j + 1; i += blockDim.x) Hc[i] = col[i];
}

// The end of an Arnoldi step in one launch: block 0 takes the Givens step,
// the other blocks form v_{j+1} = w / |w| (skipped when the gate is set: the
// second Gram-Schmidt update wrote it).  The Givens step writes |w| only when
// the gate is set, the scale reads it only when it is not, so the blocks do
// not race.
__global__ __launch_bounds__(KT) void k_scale_givens(GivensSet S, long long n, int j, int ldh) {
  const int sy = blockIdx.y;
  if (blockIdx.x == 0)
    givens_body(S.H[sy], S.h[sy], S.wnorm2[sy], S.cs[sy], S.sn[sy], S.g[sy], j, ldh, S.est[sy],
                S.h2[sy], S.gate[sy], S.wnorm2_alt[sy], S.host_out[sy]);
  else
    scale_body(S.w[sy], S.wnorm2[sy], S.v[sy], n, S.gate[sy], blockIdx.x - 1, gridDim.x - 1);
}

// y = R^{-1} g by back substitution on one thread.  For k <= TSL the upper
// triangle of R and g are first staged in LDS by the whole block, so that the
// serial chain waits on no memory round trips; larger k reads them directly.
constexpr int TSL = 40;
__device__ inline void trisolve_body(const double2* __restrict__ H, const double2* __restrict__ g,
                                     double2* __restrict__ y, int k, int ldh) {
  __shared__ double2 R[TSL * TSL];
  __shared__ double2 gs[TSL], ys[TSL];
  if (k <= TSL) {
    for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
      const int c = e / k, r = e - c * k;
      if (r <= c) R[c * TSL + r] = H[(long long)c * ldh + r];
    }
    for (int i = threadIdx.x; i < k; i += blockDim.x) gs[i] = g[i];
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int i = k - 1; i >= 0; --i) {
      double2 s = gs[i];
      for (int t = i + 1; t < k; ++t) s = cfms(R[t * TSL + i], ys[t], s);
      ys[i] = cdiv(s, R[i * TSL + i]);
      y[i] = ys[i];
    }
    return;
  }
  if (threadIdx.x != 0) return;
  for (int i = k - 1; i >= 0; --i) {
    double2 s = g[i];
    for (int t = i + 1; t < k; ++t) s = cfms(H[(long long)t * ldh + i], y[t], s);
    y[i] = cdiv(s, H[(long long)i * ldh + i]);
  }
}

// One block per right-hand side (blockIdx.x = s).
__global__ void k_trisolve(CycleSet S, int ldh) {
  const int s = blockIdx.x;
  trisolve_body(S.H[s], S.g[s], S.y[s], S.k[s], ldh);
}

__global__ __launch_bounds__(KT) void k_xupdate(CycleSet S, long long ld, long long n) {
  const int sy = blockIdx.y;
  const double2* __restrict__ Z = S.Z[sy];
  const int k = S.k[sy];
  const double2* __restrict__ y = S.y[sy];
  double2* __restrict__ x = S.x[sy];
  __shared__ double2 ys[256];
  if ((int)threadIdx.x < k) ys[threadIdx.x] = y[threadIdx.x];
  __syncthreads();
  for (long long t = (long long)blockIdx.x * KT + threadIdx.x; t < n; t += (long long)gridDim.x * KT) {
    double2 acc = x[t];
    for (int i = 0; i < k; ++i) acc = cfma(Z[(long long)i * ld + t], ys[i], acc);
    x[t] = acc;
  }
}

__global__ __launch_bounds__(KT) void k_axpy(double2* __restrict__ y, const double2* __restrict__ x,
                                             long long n) {
  for (long long t = (long long)blockIdx.x * KT + threadIdx.x; t < n; t += (long long)gridDim.x * KT) {
    double2 a = y[t], b = x[t];
    y[t] = make_double2(a.x + b.x, a.y + b.y);
  }
}

int grid_for(long long n) {
  long long g = (n + KT - 1) / KT;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace

int krylov_blocks(long long n) { return (int)((n + CHUNK - 1) / CHUNK); }

void launch_mdot(hipStream_t st, const double2* V, long long ld, int nv, const double2* w,
                 long long n, double2* partial, double* norm_partial, const int* gate) {
  STF_LAUNCH(k_mdot, dim3(krylov_blocks(n)), dim3(KT), 0, st, V, ld, nv, w, n, partial,
                     norm_partial, gate);
}

void launch_mdot_reduce(hipStream_t st, const double2* partial, int nblk, int nv, double2* h,
                        const int* gate, int stride) {
  STF_LAUNCH(k_mdot_reduce, dim3(nv), dim3(KT), 0, st, partial, nblk,
                     stride > 0 ? stride : nv, h, gate);
}

int gs_stride(int nv) { return nv <= 8 ? 8 : nv <= 16 ? 16 : nv <= 32 ? 32 : 0; }

int gs_blocks(long long n, int nv) {
  const int nvm = gs_stride(nv);
  const int ept = nvm > 0 ? 32 / nvm : 1;
  return (int)((n + (long long)KT * ept - 1) / ((long long)KT * ept));
}


void launch_gs_reduce_set(hipStream_t st, int nr, const GsRedSet& S, int nblk, int stride, int nv) {
  STF_REQUIRE(nr >= 1 && nr <= MAX_RHS, "1 to 4 right-hand sides per launch");
  STF_LAUNCH(k_gs_reduce, dim3(nv + 1, nr), dim3(KT), 0, st, S, nblk, stride, nv);
}

void launch_gs_reduce(hipStream_t st, const double2* partial, int nblk, int stride, int nv,
                      double2* h, const double* npart, double* out, const double* ref, int* gate) {
  GsRedSet S;
  S.partial[0] = partial;
  S.h[0] = h;
  S.npart[0] = npart;
  S.out[0] = out;
  S.ref[0] = ref;
  S.gate[0] = gate;
  launch_gs_reduce_set(st, 1, S, nblk, stride, nv);
}

void launch_gs_set(hipStream_t st, int mode, int nr, const GsSet& S, long long ld, int nv, long long n) {
  const int nvm = gs_stride(nv);
  STF_REQUIRE(nvm > 0 && nv >= 1, "register Gram-Schmidt pass takes 1..32 basis vectors");
  STF_REQUIRE(mode >= GS_DOT && mode <= GS_UPDATE_NORMALIZE, "unknown Gram-Schmidt pass");
  STF_REQUIRE(nr >= 1 && nr <= MAX_RHS, "1 to 4 right-hand sides per launch");
  for (int s = 0; s < nr; ++s)
    STF_REQUIRE(mode != GS_UPDATE_NORMALIZE || (S.vout[s] && S.nrm_in[s] && S.nrm_out[s]),
                "normalising pass needs its output vector and norms");
  const dim3 g(gs_blocks(n, nv), nr), b(KT);
#define STF_GS_CASE(M)                                                                        \
  if (nvm == M) {                                                                             \
    if (mode == GS_DOT)                                                                       \
      STF_LAUNCH((k_gs<M, false, true, false>), g, b, 0, st, S, ld, nv, n);           \
    else if (mode == GS_UPDATE_DOT)                                                           \
      STF_LAUNCH((k_gs<M, true, true, false>), g, b, 0, st, S, ld, nv, n);            \
    else if (mode == GS_UPDATE)                                                               \
      STF_LAUNCH((k_gs<M, true, false, false>), g, b, 0, st, S, ld, nv, n);           \
    else                                                                                      \
      STF_LAUNCH((k_gs<M, true, false, true>), g, b, 0, st, S, ld, nv, n);            \
    return;                                                                                   \
  }
  STF_GS_CASE(8)
  STF_GS_CASE(16)
  STF_GS_CASE(32)
#undef STF_GS_CASE
}

void launch_gs(hipStream_t st, int mode, const double2* V, long long ld, int nv, const double2* h,
               double2* w, long long n, double2* partial, double* norm_partial, const int* gate,
               double2* vout, const double* nrm_in, double* nrm_out) {
  GsSet S;
  S.V[0] = V;
  S.h[0] = h;
  S.w[0] = w;
  S.partial[0] = partial;
  S.npart[0] = norm_partial;
  S.gate[0] = gate;
  S.vout[0] = vout;
  S.nrm_in[0] = nrm_in;
  S.nrm_out[0] = nrm_out;
  launch_gs_set(st, mode, 1, S, ld, nv, n);
}

void launch_mupdate(hipStream_t st, const double2* V, long long ld, int nv, const double2* h,
                    double2* w, long long n, double* norm_partial, const int* gate) {
  STF_LAUNCH(k_mupdate, dim3(krylov_blocks(n)), dim3(KT), 0, st, V, ld, nv, h, w, n,
                     norm_partial, gate);
}

void launch_norm_reduce(hipStream_t st, const double* partial, int n, double* out,
                        const double* ref, int* gate, int decide) {
  STF_LAUNCH(k_norm_reduce, dim3(1), dim3(KT), 0, st, partial, n, out, ref, gate, decide);
}

void launch_hacc(hipStream_t st, double2* h1, const double2* h2, int nv, const int* gate) {
  STF_LAUNCH(k_hacc, dim3(1), dim3(256), 0, st, h1, h2, nv, gate);
}

void launch_cycle_start_set(hipStream_t st, int nr, const CycleSet& S, long long n, int glen) {
  STF_REQUIRE(nr >= 1 && nr <= MAX_RHS, "1 to 4 right-hand sides per launch");
  STF_LAUNCH(k_cycle_start, dim3(grid_for(n), nr), dim3(KT), 0, st, S, n, glen);
}


void launch_scale(hipStream_t st, const double2* w, const double* nrm2, double2* v, long long n,
                  const int* skip) {
  STF_LAUNCH(k_scale, dim3(grid_for(n)), dim3(KT), 0, st, w, nrm2, v, n, skip);
}

void launch_scale_givens_set(hipStream_t st, int nr, const GivensSet& S, long long n, int j, int ldh) {
  STF_REQUIRE(j >= 0 && j < GV, "Givens step beyond the staged column");
  STF_REQUIRE(nr >= 1 && nr <= MAX_RHS, "1 to 4 right-hand sides per launch");
  STF_LAUNCH(k_scale_givens, dim3(grid_for(n) + 1, nr), dim3(KT), 0, st, S, n, j, ldh);
}

void launch_scale_givens(hipStream_t st, const double2* w, double2* v, long long n, double2* H,
                         const double2* h, double* wnorm2, double* cs, double2* sn, double2* g,
                         int j, int ldh, double* est_out, const double2* h2, const int* gate,
                         const double* wnorm2_alt, double* host_out) {
  GivensSet S;
  S.w[0] = w;
  S.v[0] = v;
  S.H[0] = H;
  S.h[0] = h;
  S.wnorm2[0] = wnorm2;
  S.cs[0] = cs;
  S.sn[0] = sn;
  S.g[0] = g;
  S.est[0] = est_out;
  S.h2[0] = h2;
  S.gate[0] = gate;
  S.wnorm2_alt[0] = wnorm2_alt;
  S.host_out[0] = host_out;
  launch_scale_givens_set(st, 1, S, n, j, ldh);
}

void launch_axpy(hipStream_t st, double2* y, const double2* x, long long n) {
  STF_LAUNCH(k_axpy, dim3(grid_for(n)), dim3(KT), 0, st, y, x, n);
}

void launch_trisolve_set(hipStream_t st, int nr, const CycleSet& S, int ldh) {
  STF_REQUIRE(nr >= 1 && nr <= MAX_RHS, "1 to 4 right-hand sides per launch");
  STF_LAUNCH(k_trisolve, dim3(nr), dim3(64), 0, st, S, ldh);
}

void launch_xupdate_set(hipStream_t st, int nr, const CycleSet& S, long long ld, long long n) {
  STF_REQUIRE(nr >= 1 && nr <= MAX_RHS, "1 to 4 right-hand sides per launch");
  STF_LAUNCH(k_xupdate, dim3(grid_for(n), nr), dim3(KT), 0, st, S, ld, n);
}

}  // namespace stf
