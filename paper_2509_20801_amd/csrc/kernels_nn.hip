// Learned warm start: FP32 kernels of the spectral neural operator (forward,
// backward, loss, Adam) and of the tiled initial guess (features, blending).
//
// Tensors are planar, [sample][channel][y][x] with x fastest.  The spectral
// convolution keeps the modes k = 0..M-1 along x and ky = -M..M-1 along y; the
// truncated DFTs are evaluated as products with twiddle tables: the large ones
// (along x forward, along y inverse) through a batched, strided, LDS-tiled
// GEMM, the small ones (along y forward, along x inverse, the per-mode channel
// mixing) by dedicated kernels.  Gradient reductions are per-block partial
// sums added in a fixed order, so training is deterministic.
#include <cmath>

#include "stf_internal.h"

namespace stf {

namespace {

constexpr int NNT = 256;

__device__ inline float gelu_f(float x) {
  const float c = 0.7978845608028654f;
  return 0.5f * x * (1.0f + tanhf(c * (x + 0.044715f * x * x * x)));
}

__device__ inline float gelu_df(float x) {
  const float c = 0.7978845608028654f;
  const float t = tanhf(c * (x + 0.044715f * x * x * x));
  return 0.5f * (1.0f + t) + 0.5f * x * (1.0f - t * t) * c * (1.0f + 3.0f * 0.044715f * x * x);
}

// ---------------------------------------------------------------------------
// C[b] = alpha A[b] B[b] + beta C[b], A (M x K), B (K x N), arbitrary strides.
// TM x TN output tile per 256-thread workgroup (64 x 64, or 128 x 32 for the
// narrow products of the x transform), 4 x 4 per thread, K staged in LDS 16 at
// a time.  Tiles are loaded along whichever index is contiguous in memory, so
// that consecutive threads read consecutive addresses.
// ---------------------------------------------------------------------------
struct GemmArgs {
  const float* A;
  const float* B;
  float* C;
  int M, N, K;
  long long sAb, sAm, sAk, sBb, sBk, sBn, sCb, sCm, sCn;
  float alpha, beta;
};

template <int TM, int TN>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
  constexpr int TK = 16, RX = TN / 4, RY = TM / 4;         // threads per row / column of the tile
  static_assert(RX * RY == 256, "4 x 4 outputs per thread");
  __shared__ float As[TK][TM + 4];
  __shared__ float Bs[TK][TN + 4];
  const int tid = threadIdx.x, tx = tid % RX, ty = tid / RX;
  const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN, b = blockIdx.z;
  const float* A = g.A + b * g.sAb;
  const float* Bm = g.B + b * g.sBb;
  const bool a_k_fast = g.sAk == 1, b_n_fast = g.sBn == 1;
  float acc[4][4] = {};
  for (int k0 = 0; k0 < g.K; k0 += TK) {
    for (int t = tid; t < TM * TK; t += 256) {
      const int mm = a_k_fast ? t / TK : t % TM, kk = a_k_fast ? t % TK : t / TM;
      const int m = m0 + mm, k = k0 + kk;
      As[kk][mm] = (m < g.M && k < g.K) ? A[m * g.sAm + k * g.sAk] : 0.0f;
    }
    for (int t = tid; t < TN * TK; t += 256) {
      const int nn = b_n_fast ? t % TN : t / TK, kk = b_n_fast ? t / TN : t % TK;
      const int n = n0 + nn, k = k0 + kk;
      Bs[kk][nn] = (n < g.N && k < g.K) ? Bm[k * g.sBk + n * g.sBn] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TK; ++kk) {
      float a[4], bb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + RY * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) bb[j] = Bs[kk][tx + RX * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], bb[j], acc[i][j]);
    }
    __syncthreads();
  }
  float* C = g.C + b * g.sCb;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = m0 + ty + RY * i;
    if (m >= g.M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = n0 + tx + RX * j;
      if (n >= g.N) continue;
      float* c = C + m * g.sCm + n * g.sCn;
      *c = g.alpha * acc[i][j] + (g.beta != 0.0f ? g.beta * *c : 0.0f);
    }
  }
}

// ---------------------------------------------------------------------------
// The x transform of every row: a tall A (M x K, K <= 256) times a narrow B
// (K x N, N <= 32) on the FP32 matrix cores.  B is held whole in LDS; each
// workgroup streams 64 rows of A through LDS 64 columns at a time (16-byte
// loads along the rows when VEC: every row start 16-byte aligned, K % 4 = 0),
// and each wavefront forms a 16 x 32 block of C as two 16x16x4 products per
// step of 4 in K.  Lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16];
// output (i, j) of a 16 x 16 tile is in lane j + 16 (i / 4), register i % 4.
// ---------------------------------------------------------------------------
template <bool VEC>
__global__ __launch_bounds__(256) void k_gemm_tall(GemmArgs g) {
  typedef float V4 __attribute__((ext_vector_type(4)));
  __shared__ float Bs[256][33];
  __shared__ float As[64][65];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, b = blockIdx.z;
  const float* A = g.A + b * g.sAb;
  const float* Bm = g.B + b * g.sBb;
  // B whole (rows beyond K zero, read by the last step of 4): 32 entries per
  // thread, loaded in batches of 16 (all loads of a batch in flight before
  // any is stored)
  for (int t0 = 0; t0 < 256 * 32; t0 += 16 * 256) {
    float v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int t = t0 + u * 256 + tid, k = t >> 5, n = t & 31;
      v[u] = (k < g.K && n < g.N) ? Bm[k * g.sBk + n * g.sBn] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int t = t0 + u * 256 + tid;
      Bs[t >> 5][t & 31] = v[u];
    }
  }
  const int m0 = blockIdx.x * 64;
  const int l16 = lane & 15, lk = lane >> 4, wr = wv * 16;
  V4 acc0 = {0.0f, 0.0f, 0.0f, 0.0f}, acc1 = {0.0f, 0.0f, 0.0f, 0.0f};
  V4 acc2 = {0.0f, 0.0f, 0.0f, 0.0f}, acc3 = {0.0f, 0.0f, 0.0f, 0.0f};
  for (int k0 = 0; k0 < g.K; k0 += 64) {
    __syncthreads();
    // 64 x 64 chunk of A: four 4-entry pieces per thread, all in flight at once
    float v[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int t = u * 256 + tid, rr = t >> 4, c4 = (t & 15) * 4;
      const int m = m0 + rr, k = k0 + c4;
#pragma unroll
      for (int e = 0; e < 4; ++e) v[u][e] = 0.0f;
      if (m < g.M) {
        const float* src = A + m * g.sAm + (long long)k * g.sAk;
        if (VEC && k + 3 < g.K) {
          const float4 x = *reinterpret_cast<const float4*>(src);
          v[u][0] = x.x; v[u][1] = x.y; v[u][2] = x.z; v[u][3] = x.w;
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e) v[u][e] = k + e < g.K ? src[e * g.sAk] : 0.0f;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int t = u * 256 + tid, rr = t >> 4, c4 = (t & 15) * 4;
#pragma unroll
      for (int e = 0; e < 4; ++e) As[rr][c4 + e] = v[u][e];
    }
    __syncthreads();
    const int kw = min(64, g.K - k0);             // columns beyond K were stored as zeros
    // two steps of 4 at a time into separate accumulators: four independent chains
    for (int kk = 0; kk < kw; kk += 8) {
      const float a = As[wr + l16][kk + lk], a2 = As[wr + l16][kk + 4 + lk];
      const float b0 = Bs[k0 + kk + lk][l16], b1 = Bs[k0 + kk + lk][16 + l16];
      const float b2 = Bs[k0 + kk + 4 + lk][l16], b3 = Bs[k0 + kk + 4 + lk][16 + l16];
      // transposed products (B^T A^T): lane (l16, lk) receives
      // C[wr + l16][16 j + 4 lk + v], four consecutive columns per lane
      acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(b0, a, acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(b1, a, acc1, 0, 0, 0);
      acc2 = __builtin_amdgcn_mfma_f32_16x16x4f32(b2, a2, acc2, 0, 0, 0);
      acc3 = __builtin_amdgcn_mfma_f32_16x16x4f32(b3, a2, acc3, 0, 0, 0);
    }
  }
  acc0 += acc2;
  acc1 += acc3;
  float* C = g.C + b * g.sCb;
  const int m = m0 + wr + l16;
  if (m >= g.M) return;
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int n = 16 * j + 4 * lk + v;
      if (n < g.N) {
        float* c = C + m * g.sCm + n * g.sCn;
        const float x = j == 0 ? acc0[v] : acc1[v];
        *c = g.alpha * x + (g.beta != 0.0f ? g.beta * *c : 0.0f);
      }
    }
}

// ---------------------------------------------------------------------------
// The inverse x transform: C (M x N) = alpha A (M x K) B (K x N) + beta C per
// batch entry for K <= 64 on the FP32 matrix cores: a 64 x 64 tile of C per
// workgroup, 32 x 32 per wavefront as 2 x 2 16x16x4 products, K staged in LDS
// whole.  Lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]; output
// (i, j) of a 16 x 16 tile is in lane j + 16 (i / 4), register i % 4.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_gemm_mfma(GemmArgs g) {
  typedef float V4 __attribute__((ext_vector_type(4)));
  __shared__ float As[64][65];          // [k][m]
  __shared__ float Bs[64][65];          // [k][n]
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64, b = blockIdx.z;
  const float* A = g.A + b * g.sAb;
  const float* Bm = g.B + b * g.sBb;
  // A along k when its rows are contiguous, else along m; B along n when its
  // rows are contiguous, else along k; sixteen entries of each per thread, all
  // in flight before any is stored.
  const bool ak = g.sAk == 1, bn = g.sBn == 1;
  float va[16], vb[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int t = u * 256 + tid;
    const int mm = ak ? t >> 6 : t & 63, kk = ak ? t & 63 : t >> 6;
    const int m = m0 + mm;
    va[u] = (m < g.M && kk < g.K) ? A[m * g.sAm + kk * g.sAk] : 0.0f;
    const int nn = bn ? t & 63 : t >> 6, kb = bn ? t >> 6 : t & 63;
    const int n = n0 + nn;
    vb[u] = (n < g.N && kb < g.K) ? Bm[kb * g.sBk + n * g.sBn] : 0.0f;
  }
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int t = u * 256 + tid;
    As[ak ? t & 63 : t >> 6][ak ? t >> 6 : t & 63] = va[u];
    Bs[bn ? t >> 6 : t & 63][bn ? t & 63 : t >> 6] = vb[u];
  }
  __syncthreads();
  const int wm = (wv >> 1) * 32, wn = (wv & 1) * 32;
  const int l16 = lane & 15, lk = lane >> 4;
  V4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = V4{0.0f, 0.0f, 0.0f, 0.0f};
  for (int k0 = 0; k0 < g.K; k0 += 4) {
    const int k = k0 + lk;
    const float a0 = As[k][wm + l16], a1 = As[k][wm + 16 + l16];
    const float b0 = Bs[k][wn + l16], b1 = Bs[k][wn + 16 + l16];
    acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
  }
  float* C = g.C + b * g.sCb;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = m0 + wm + 16 * i + 4 * lk + v, n = n0 + wn + 16 * j + l16;
        if (m < g.M && n < g.N) {
          float* c = C + m * g.sCm + n * g.sCn;
          *c = g.alpha * acc[i][j][v] + (g.beta != 0.0f ? g.beta * *c : 0.0f);
        }
      }
}

// ---------------------------------------------------------------------------
// The inverse transform of one plane in one pass: the x inverse
// S[a][x] = sum_k w_k G[a][k] exp(+2 pi i k x / n) (w_k = 1, 2, 2, ... when
// weighted) formed in LDS as rows [Re S; Im S] (4M x n), then the y inverse
// out = alpha Ainv S + beta out (Ainv: n x 4M, rows contiguous) on the FP32
// matrix cores, 16 x 16 tiles of out, a wavefront per 16-row block at a time
// with its rows of Ainv held in registers across the column blocks.  n is a
// multiple of 16 (at most 1024), 4M <= 88; out 16-byte aligned with npix a
// multiple of 4.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_spec_inv(const float2* __restrict__ G,
                                                  const float2* __restrict__ ex, int n, int M,
                                                  int weighted, const float* __restrict__ ainv,
                                                  float alpha, float beta, float* __restrict__ out,
                                                  long long npix) {
  typedef float V4 __attribute__((ext_vector_type(4)));
  extern __shared__ float Ss[];                  // 4M x (n + 16): rows 16 banks apart
  __shared__ float2 Gs[2 * 22 * 22];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int plane = blockIdx.x, ld = n + 16, K = 4 * M;
  const float2* Gp = G + (long long)plane * 2 * M * M;
  for (int t = tid; t < 2 * M * M; t += 256) {
    float2 v = Gp[t];
    if (weighted && t % M > 0) v = make_float2(2.0f * v.x, 2.0f * v.y);
    Gs[t] = v;
  }
  __syncthreads();
  // S: thread per column x, its M twiddles in registers
  for (int x = tid; x < n; x += 256) {
    float2 w[22];
#pragma unroll
    for (int k = 0; k < 22; ++k) w[k] = k < M ? ex[(long long)k * n + x] : make_float2(0.0f, 0.0f);
    for (int a = 0; a < 2 * M; ++a) {
      float re = 0.0f, im = 0.0f;
#pragma unroll
      for (int k = 0; k < 22; ++k)
        if (k < M) {
          const float2 gv = Gs[a * M + k];
          re = fmaf(gv.x, w[k].x, fmaf(-gv.y, w[k].y, re));
          im = fmaf(gv.x, w[k].y, fmaf(gv.y, w[k].x, im));
        }
      Ss[a * ld + x] = re;
      Ss[(2 * M + a) * ld + x] = im;
    }
  }
  __syncthreads();
  const int l16 = lane & 15, lk = lane >> 4, nb = n / 16;
  float* op = out + (long long)plane * npix;
  for (int yb = wv; yb < nb; yb += 4) {
    float av[22];                                // Ainv[yb*16 + l16][4 s + lk], s < K / 4
#pragma unroll
    for (int s4 = 0; s4 < 22; ++s4)
      av[s4] = 4 * s4 < K ? ainv[(long long)(yb * 16 + l16) * K + 4 * s4 + lk] : 0.0f;
    // four column blocks at a time: four independent accumulation chains
    for (int xb0 = 0; xb0 < nb; xb0 += 4) {
      V4 acc[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[j] = V4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int s4 = 0; s4 < 22; ++s4)
        if (4 * s4 < K) {
          float bv[4];
#pragma unroll
          for (int j = 0; j < 4; ++j)
            bv[j] = xb0 + j < nb ? Ss[(4 * s4 + lk) * ld + (xb0 + j) * 16 + l16] : 0.0f;
          // the transposed product (S^T Ainv^T): lane (l16, lk) receives
          // out[yb*16 + l16][x0 + 4 lk + v], four consecutive x per lane
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(bv[j], av[s4], acc[j], 0, 0, 0);
        }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (xb0 + j >= nb) continue;
        float4* c = reinterpret_cast<float4*>(op + (long long)(yb * 16 + l16) * n + (xb0 + j) * 16 + 4 * lk);
        float4 r = make_float4(alpha * acc[j][0], alpha * acc[j][1], alpha * acc[j][2], alpha * acc[j][3]);
        if (beta != 0.0f) {
          const float4 o = *c;
          r.x += beta * o.x; r.y += beta * o.y; r.z += beta * o.z; r.w += beta * o.w;
        }
        *c = r;
      }
    }
  }
}

// The same for the compiled tile side NN and mode count MM (the trained
// network's n = 256, M = 16): every LDS offset an immediate, loops unrolled.
template <int NN, int MM>
__global__ __launch_bounds__(256) void k_spec_inv_t(const float2* __restrict__ G,
                                                    const float2* __restrict__ ex, int weighted,
                                                    const float* __restrict__ ainv, float alpha,
                                                    float beta, float* __restrict__ out, long long npix) {
  typedef float V4 __attribute__((ext_vector_type(4)));
  constexpr int LD = NN + 16, K = 4 * MM, NB = NN / 16;
  static_assert(NN % 64 == 0 && NN <= 256, "a column per thread, four column blocks per group");
  extern __shared__ float Ss[];                  // K x LD
  __shared__ float2 Gs[2 * MM * MM];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int plane = blockIdx.x;
  const float2* Gp = G + (long long)plane * 2 * MM * MM;
  for (int t = tid; t < 2 * MM * MM; t += 256) {
    float2 v = Gp[t];
    if (weighted && t % MM > 0) v = make_float2(2.0f * v.x, 2.0f * v.y);
    Gs[t] = v;
  }
  __syncthreads();
  if (tid < NN) {
    const int x = tid;
    float2 w[MM];
#pragma unroll
    for (int k = 0; k < MM; ++k) w[k] = ex[k * NN + x];
#pragma unroll 4
    for (int a = 0; a < 2 * MM; ++a) {
      float re = 0.0f, im = 0.0f;
#pragma unroll
      for (int k = 0; k < MM; ++k) {
        const float2 gv = Gs[a * MM + k];
        re = fmaf(gv.x, w[k].x, fmaf(-gv.y, w[k].y, re));
        im = fmaf(gv.x, w[k].y, fmaf(gv.y, w[k].x, im));
      }
      Ss[a * LD + x] = re;
      Ss[(2 * MM + a) * LD + x] = im;
    }
  }
  __syncthreads();
  const int l16 = lane & 15, lk = lane >> 4;
  float* op = out + (long long)plane * npix;
  const float* sb = Ss + lk * LD + l16;
  for (int yb = wv; yb < NB; yb += 4) {
    float av[K / 4];
    const float* ar = ainv + (yb * 16 + l16) * K + lk;
#pragma unroll
    for (int s4 = 0; s4 < K / 4; ++s4) av[s4] = ar[4 * s4];
    float* orow = op + (long long)(yb * 16 + l16) * NN + 4 * lk;
    for (int xb0 = 0; xb0 < NB; xb0 += 4) {
      V4 acc[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[j] = V4{0.0f, 0.0f, 0.0f, 0.0f};
      const float* sx = sb + xb0 * 16;
#pragma unroll
      for (int s4 = 0; s4 < K / 4; ++s4) {
        float bv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) bv[j] = sx[4 * s4 * LD + j * 16];
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(bv[j], av[s4], acc[j], 0, 0, 0);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        float4* c = reinterpret_cast<float4*>(orow + (xb0 + j) * 16);
        float4 r = make_float4(alpha * acc[j][0], alpha * acc[j][1], alpha * acc[j][2], alpha * acc[j][3]);
        if (beta != 0.0f) {
          const float4 o = *c;
          r.x += beta * o.x; r.y += beta * o.y; r.z += beta * o.z; r.w += beta * o.w;
        }
        *c = r;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Truncated DFT along y of one plane: H[a, k] = s_k sum_y Ey[a, y] T[y, k],
// T row y = [Re (M) | Im (M)] of the x transform, Ey = exp(-2 pi i ky(a) y / n).
// s_k = 1 (forward) or w_k / n^2 (gradient through the inverse transform).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(NNT) void k_dft_y(const float* __restrict__ T,
                                               const float2* __restrict__ ey, int n, int M,
                                               int grad_scale, float2* __restrict__ H) {
  extern __shared__ float Ts[];                  // n x 2M
  const int plane = blockIdx.x;
  const float* Tp = T + (long long)plane * n * 2 * M;
  // the plane into LDS, sixteen loads per thread in flight at a time
  for (int t0 = 0; t0 < n * 2 * M; t0 += 16 * NNT) {
    float v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int t = t0 + u * NNT + threadIdx.x;
      v[u] = t < n * 2 * M ? Tp[t] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int t = t0 + u * NNT + threadIdx.x;
      if (t < n * 2 * M) Ts[t] = v[u];
    }
  }
  __syncthreads();
  const float inv = 1.0f / ((float)n * (float)n);
  // Twiddles ey[a][y] staged in LDS YC columns at a time (after the plane).
  constexpr int YC = 64;
  float2* Es = reinterpret_cast<float2*>(Ts + n * 2 * M);   // 2M x YC
  constexpr int OPT = 4;                                       // outputs per thread (2M M <= OPT NNT)
  float re[OPT] = {}, im[OPT] = {};
  for (int y0 = 0; y0 < n; y0 += YC) {
    const int yc = min(YC, n - y0);
    __syncthreads();
    for (int t0 = 0; t0 < 2 * M * YC; t0 += 8 * NNT) {
      float2 v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int t = t0 + u * NNT + threadIdx.x, a = t / YC, y = t - a * YC;
        v[u] = (a < 2 * M && y < yc) ? ey[(long long)a * n + y0 + y] : make_float2(0.0f, 0.0f);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int t = t0 + u * NNT + threadIdx.x;
        if (t < 2 * M * YC) Es[t] = v[u];
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < OPT; ++j) {
      const int o = threadIdx.x + j * NNT;
      if (o >= 2 * M * M) continue;
      const int a = o / M, k = o - a * M;
      for (int y = 0; y < yc; ++y) {
        const float2 w = Es[a * YC + y];
        const float tr = Ts[(y0 + y) * 2 * M + k], ti = Ts[(y0 + y) * 2 * M + M + k];
        re[j] = fmaf(w.x, tr, fmaf(-w.y, ti, re[j]));
        im[j] = fmaf(w.x, ti, fmaf(w.y, tr, im[j]));
      }
    }
  }
  for (int j = 0; j < OPT; ++j) {
    const int o = threadIdx.x + j * NNT;
    if (o >= 2 * M * M) continue;
    const int k = o % M;
    float s = 1.0f;
    if (grad_scale) s = (k == 0 ? 1.0f : 2.0f) * inv;
    H[(long long)plane * 2 * M * M + o] = make_float2(s * re[j], s * im[j]);
  }
}

// Inverse along x of one plane: S[a, x] = sum_k w_k G[a, k] exp(+2 pi i k x / n)
// (w_k = 1, 2, 2, ... when weighted, else 1), stored planar: Re rows 0..2M-1,
// Im rows 2M..4M-1, each of n entries.
__global__ __launch_bounds__(NNT) void k_dft_x_inv(const float2* __restrict__ G,
                                                   const float2* __restrict__ ex, int n, int M,
                                                   int weighted, float* __restrict__ S) {
  extern __shared__ float2 Gs[];                 // 2M x M
  const int plane = blockIdx.y;
  const float2* Gp = G + (long long)plane * 2 * M * M;
  for (int t = threadIdx.x; t < 2 * M * M; t += NNT) Gs[t] = Gp[t];
  __syncthreads();
  const int o = blockIdx.x * NNT + threadIdx.x;
  if (o >= 2 * M * n) return;
  const int a = o / n, x = o - a * n;
  float re = 0.0f, im = 0.0f;
  for (int k0 = 0; k0 < M; k0 += 8) {
    float2 w[8];                                 // exp(+2 pi i k x / n), eight per round trip
#pragma unroll
    for (int u = 0; u < 8; ++u)
      w[u] = k0 + u < M ? ex[(long long)(k0 + u) * n + x] : make_float2(0.0f, 0.0f);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int k = k0 + u;
      if (k < M) {
        float2 gv = Gs[a * M + k];
        if (weighted && k > 0) gv = make_float2(2.0f * gv.x, 2.0f * gv.y);
        re = fmaf(gv.x, w[u].x, fmaf(-gv.y, w[u].y, re));
        im = fmaf(gv.x, w[u].y, fmaf(gv.y, w[u].x, im));
      }
    }
  }
  float* Sp = S + (long long)plane * 4 * M * n;
  Sp[(long long)a * n + x] = re;
  Sp[(long long)(2 * M + a) * n + x] = im;
}

// G[b, o, mode] = sum_i R[i, o, mode] H[b, i, mode].
__global__ __launch_bounds__(NNT) void k_mix_fwd(const float2* __restrict__ H,
                                                 const float* __restrict__ Rre,
                                                 const float* __restrict__ Rim, int B, int W,
                                                 int NM, float2* __restrict__ G) {
  const long long t = (long long)blockIdx.x * NNT + threadIdx.x;
  if (t >= (long long)B * W * NM) return;
  const int mode = (int)(t % NM);
  const int o = (int)((t / NM) % W);
  const int b = (int)(t / ((long long)NM * W));
  float re = 0.0f, im = 0.0f;
  for (int i = 0; i < W; ++i) {
    const long long ri = ((long long)i * W + o) * NM + mode;
    const float rr = Rre[ri], rim = Rim[ri];
    const float2 h = H[((long long)b * W + i) * NM + mode];
    re = fmaf(rr, h.x, fmaf(-rim, h.y, re));
    im = fmaf(rr, h.y, fmaf(rim, h.x, im));
  }
  G[t] = make_float2(re, im);
}

// dH[b, i, mode] = sum_o conj(R[i, o, mode]) dG[b, o, mode].
__global__ __launch_bounds__(NNT) void k_mix_bwd_h(const float2* __restrict__ dG,
                                                   const float* __restrict__ Rre,
                                                   const float* __restrict__ Rim, int B, int W,
                                                   int NM, float2* __restrict__ dH) {
  const long long t = (long long)blockIdx.x * NNT + threadIdx.x;
  if (t >= (long long)B * W * NM) return;
  const int mode = (int)(t % NM);
  const int i = (int)((t / NM) % W);
  const int b = (int)(t / ((long long)NM * W));
  float re = 0.0f, im = 0.0f;
  for (int o = 0; o < W; ++o) {
    const long long ri = ((long long)i * W + o) * NM + mode;
    const float rr = Rre[ri], rim = Rim[ri];
    const float2 d = dG[((long long)b * W + o) * NM + mode];
    re = fmaf(rr, d.x, fmaf(rim, d.y, re));       // conj(R) d
    im = fmaf(rr, d.y, fmaf(-rim, d.x, im));
  }
  dH[t] = make_float2(re, im);
}

// dR[i, o, mode] = sum_b conj(H[b, i, mode]) dG[b, o, mode] (Re and Im blocks).
__global__ __launch_bounds__(NNT) void k_mix_bwd_r(const float2* __restrict__ H,
                                                   const float2* __restrict__ dG, int B, int W,
                                                   int NM, float* __restrict__ dRre,
                                                   float* __restrict__ dRim) {
  const long long t = (long long)blockIdx.x * NNT + threadIdx.x;
  if (t >= (long long)W * W * NM) return;
  const int mode = (int)(t % NM);
  const int o = (int)((t / NM) % W);
  const int i = (int)(t / ((long long)NM * W));
  float re = 0.0f, im = 0.0f;
  for (int b = 0; b < B; ++b) {
    const float2 h = H[((long long)b * W + i) * NM + mode];
    const float2 d = dG[((long long)b * W + o) * NM + mode];
    re = fmaf(h.x, d.x, fmaf(h.y, d.y, re));
    im = fmaf(h.x, d.y, fmaf(-h.y, d.x, im));
  }
  dRre[t] = re;
  dRim[t] = im;
}

// The x-inverse rows S (4M x NN per plane: Re rows, then Im rows) of the
// compiled shape, a thread per column that loads its twiddles once for all 2M
// rows (the first phase of k_spec_inv_t, written to memory).
template <int NN, int MM>
__global__ __launch_bounds__(NN) void k_spec_rows_t(const float2* __restrict__ G,
                                                    const float2* __restrict__ ex,
                                                    float* __restrict__ S) {
  __shared__ float2 Gs[2 * MM * MM];
  const int x = threadIdx.x, plane = blockIdx.x;
  const float2* Gp = G + (long long)plane * 2 * MM * MM;
  for (int t = x; t < 2 * MM * MM; t += NN) {
    float2 v = Gp[t];
    if (t % MM > 0) v = make_float2(2.0f * v.x, 2.0f * v.y);
    Gs[t] = v;
  }
  __syncthreads();
  float2 w[MM];
#pragma unroll
  for (int k = 0; k < MM; ++k) w[k] = ex[k * NN + x];
  float* Sp = S + (long long)plane * 4 * MM * NN;
#pragma unroll 4
  for (int a = 0; a < 2 * MM; ++a) {
    float re = 0.0f, im = 0.0f;
#pragma unroll
    for (int k = 0; k < MM; ++k) {
      const float2 gv = Gs[a * MM + k];
      re = fmaf(gv.x, w[k].x, fmaf(-gv.y, w[k].y, re));
      im = fmaf(gv.x, w[k].y, fmaf(gv.y, w[k].x, im));
    }
    Sp[a * NN + x] = re;
    Sp[(2 * MM + a) * NN + x] = im;
  }
}

// ---------------------------------------------------------------------------
// Inference of a layer of the compiled shape (n = NN, M = MM, width WD) with
// the spectral branch and the pointwise part in one pass: for a 16 x 16 pixel
// block of one tile, every output channel o gets g_o = alpha Ainv S_o (the y
// inverse transform of the rows S_o that k_dft_x_inv wrote, on the FP32 matrix
// cores with the operand layout and summation order of k_spec_inv_t), then
// out_o = act(bias_o + sum_i W[o, i] h_i + g_o) in the order of k_pw_fwd; g
// never goes to memory.  Workgroup: 16 rows of one tile, four 16-column blocks
// (a wavefront each); each lane ends with 4 consecutive pixels of one row.
// ---------------------------------------------------------------------------
template <int NN, int MM, int WD, bool ACT>
__global__ __launch_bounds__(256) void k_spec_pw_t(const float* __restrict__ S,
                                                   const float* __restrict__ ainv, float alpha,
                                                   const float* __restrict__ hin,
                                                   const float* __restrict__ Wm,
                                                   const float* __restrict__ bias, long long npix,
                                                   float* __restrict__ out) {
  typedef float V4 __attribute__((ext_vector_type(4)));
  constexpr int K = 4 * MM;
  static_assert(NN % 64 == 0 && K % 4 == 0, "four 16-column blocks per workgroup");
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int l16 = lane & 15, lk = lane >> 4;
  const int b = blockIdx.z, yb = blockIdx.y, xb = blockIdx.x * 4 + wv;
  // the input channels of this lane's four pixels first: their loads overlap
  // the products below
  const long long pix = (long long)(yb * 16 + l16) * NN + xb * 16 + 4 * lk;
  float4 hv[WD];
#pragma unroll
  for (int i = 0; i < WD; ++i) hv[i] = *reinterpret_cast<const float4*>(hin + ((long long)b * WD + i) * npix + pix);
  float av[K / 4];
  const float* ar = ainv + (yb * 16 + l16) * K + lk;
#pragma unroll
  for (int s4 = 0; s4 < K / 4; ++s4) av[s4] = ar[4 * s4];
  V4 acc[WD];
#pragma unroll
  for (int o = 0; o < WD; ++o) {
    const float* sp = S + ((long long)b * WD + o) * K * NN + (long long)lk * NN + xb * 16 + l16;
    float bv[K / 4];
#pragma unroll
    for (int s4 = 0; s4 < K / 4; ++s4) bv[s4] = sp[(long long)4 * s4 * NN];
    acc[o] = V4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int s4 = 0; s4 < K / 4; ++s4) acc[o] = __builtin_amdgcn_mfma_f32_16x16x4f32(bv[s4], av[s4], acc[o], 0, 0, 0);
  }
#pragma unroll
  for (int o = 0; o < WD; ++o) {
    float r[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      float sacc = bias[o];
#pragma unroll
      for (int i = 0; i < WD; ++i) {
        const float hi = v == 0 ? hv[i].x : v == 1 ? hv[i].y : v == 2 ? hv[i].z : hv[i].w;
        sacc = fmaf(Wm[o * WD + i], hi, sacc);
      }
      sacc += alpha * acc[o][v];
      r[v] = ACT ? gelu_f(sacc) : sacc;
    }
    *reinterpret_cast<float4*>(out + ((long long)b * WD + o) * npix + pix) = make_float4(r[0], r[1], r[2], r[3]);
  }
}

// ---------------------------------------------------------------------------
// Pointwise channel mixing, one thread per pixel:
//   pre[o] = sum_i Wm[o, i] in[i] + bias[o] (+ add[o]);  out = ACT ? gelu(pre) : pre.
// ---------------------------------------------------------------------------
template <int CI, int CO, bool ACT>
__global__ __launch_bounds__(NNT) void k_pw_fwd(const float* __restrict__ in,
                                                const float* __restrict__ Wm,
                                                const float* __restrict__ bias,
                                                const float* __restrict__ add, long long npix,
                                                int B, float* __restrict__ pre,
                                                float* __restrict__ out) {
  const long long t = (long long)blockIdx.x * NNT + threadIdx.x;
  if (t >= npix * B) return;
  const long long b = t / npix, p = t - b * npix;
  float x[CI];
#pragma unroll
  for (int i = 0; i < CI; ++i) x[i] = in[(b * CI + i) * npix + p];
#pragma unroll
  for (int o = 0; o < CO; ++o) {
    float s = bias[o];
#pragma unroll
    for (int i = 0; i < CI; ++i) s = fmaf(Wm[o * CI + i], x[i], s);
    const long long oi = (b * CO + o) * npix + p;
    if (add) s += add[oi];
    if (ACT) {
      if (pre) pre[oi] = s;          // kept for the backward pass only
      out[oi] = gelu_f(s);
    } else {
      out[oi] = s;
    }
  }
}

// Backward of k_pw_fwd over tiles of 64 pixels (one sample at a time):
//   dpre = ACT ? dout * gelu'(pre) : dout   (stored when dpre_out is given)
//   din[i] = sum_o Wm[o, i] dpre[o]          (when din is given)
//   partial[blk] = [sum dpre[o] in[i] (CO x CI), sum dpre[o] (CO)] over the block's tiles.
template <int CI, int CO, bool ACT>
__global__ __launch_bounds__(NNT) void k_pw_bwd(const float* __restrict__ dout,
                                                const float* __restrict__ pre,
                                                const float* __restrict__ in,
                                                const float* __restrict__ Wm, long long npix,
                                                int B, float* __restrict__ dpre_out,
                                                float* __restrict__ din,
                                                float* __restrict__ partial) {
  constexpr int P = 64;
  __shared__ float sd[CO][P];
  __shared__ float si[CI][P];
  const int tid = threadIdx.x;
  const long long ntile = (npix + P - 1) / P * B;
  float accw[(CO * CI + NNT - 1) / NNT] = {};
  float accb = 0.0f;
  for (long long tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
    const long long b = tile / ((npix + P - 1) / P);
    const long long p0 = (tile - b * ((npix + P - 1) / P)) * P;
    __syncthreads();
    for (int t = tid; t < CO * P; t += NNT) {
      const int o = t / P, j = t % P;
      const long long p = p0 + j;
      float d = 0.0f;
      if (p < npix) {
        const long long oi = (b * CO + o) * npix + p;
        d = dout[oi];
        if (ACT) d *= gelu_df(pre[oi]);
        if (dpre_out) dpre_out[oi] = d;
      }
      sd[o][j] = d;
    }
    for (int t = tid; t < CI * P; t += NNT) {
      const int i = t / P, j = t % P;
      const long long p = p0 + j;
      si[i][j] = p < npix ? in[(b * CI + i) * npix + p] : 0.0f;
    }
    __syncthreads();
    if (din) {
      for (int t = tid; t < CI * P; t += NNT) {
        const int i = t / P, j = t % P;
        const long long p = p0 + j;
        if (p >= npix) continue;
        float s = 0.0f;
#pragma unroll
        for (int o = 0; o < CO; ++o) s = fmaf(Wm[o * CI + i], sd[o][j], s);
        din[(b * CI + i) * npix + p] = s;
      }
    }
#pragma unroll
    for (int q = 0; q < (CO * CI + NNT - 1) / NNT; ++q) {
      const int t = tid + q * NNT;
      if (t < CO * CI) {
        const int o = t / CI, i = t % CI;
        float s = 0.0f;
        for (int j = 0; j < P; ++j) s = fmaf(sd[o][j], si[i][j], s);
        accw[q] += s;
      }
    }
    if (tid < CO) {
      float s = 0.0f;
      for (int j = 0; j < P; ++j) s += sd[tid][j];
      accb += s;
    }
  }
  float* part = partial + (long long)blockIdx.x * (CO * CI + CO);
#pragma unroll
  for (int q = 0; q < (CO * CI + NNT - 1) / NNT; ++q) {
    const int t = tid + q * NNT;
    if (t < CO * CI) part[t] = accw[q];
  }
  if (tid < CO) part[CO * CI + tid] = accb;
}

// out[j] = sum over blocks of partial[blk * stride + j], blocks in order.
__global__ __launch_bounds__(NNT) void k_sum_partials(const float* __restrict__ partial, int nblk,
                                                      int stride, int count, float* __restrict__ out) {
  const int j = blockIdx.x * NNT + threadIdx.x;
  if (j >= count) return;
  float s = 0.0f;
  for (int b = 0; b < nblk; ++b) s += partial[(long long)b * stride + j];
  out[j] = s;
}

// Per-sample sums of (y - t)^2 and t^2: partial[(b * nblk + blk) * 2 + {0, 1}].
__global__ __launch_bounds__(NNT) void k_loss_partial(const float* __restrict__ y,
                                                      const float* __restrict__ t, long long per,
                                                      int nblk, double* __restrict__ partial) {
  __shared__ double s0[NNT], s1[NNT];
  const int b = blockIdx.y, blk = blockIdx.x;
  double a0 = 0.0, a1 = 0.0;
  for (long long i = (long long)blk * NNT + threadIdx.x; i < per; i += (long long)nblk * NNT) {
    const double d = (double)y[b * per + i] - (double)t[b * per + i];
    const double tv = t[b * per + i];
    a0 += d * d;
    a1 += tv * tv;
  }
  s0[threadIdx.x] = a0;
  s1[threadIdx.x] = a1;
  __syncthreads();
  for (int s = NNT / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      s0[threadIdx.x] += s0[threadIdx.x + s];
      s1[threadIdx.x] += s1[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[((long long)b * nblk + blk) * 2] = s0[0];
    partial[((long long)b * nblk + blk) * 2 + 1] = s1[0];
  }
}

// loss = mean_b num_b / den_b; den[b] = den_b (one thread).
__global__ void k_loss_final(const double* __restrict__ partial, int B, int nblk,
                             double* __restrict__ den, double* __restrict__ loss) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double L = 0.0;
  for (int b = 0; b < B; ++b) {
    double n0 = 0.0, d0 = 0.0;
    for (int k = 0; k < nblk; ++k) {
      n0 += partial[((long long)b * nblk + k) * 2];
      d0 += partial[((long long)b * nblk + k) * 2 + 1];
    }
    den[b] = d0;
    L += n0 / d0;
  }
  *loss = L / B;
}

// dy = 2 (y - t) / (B den_b).
__global__ __launch_bounds__(NNT) void k_loss_grad(const float* __restrict__ y,
                                                   const float* __restrict__ t,
                                                   const double* __restrict__ den, long long per,
                                                   int B, float* __restrict__ dy) {
  const long long i = (long long)blockIdx.x * NNT + threadIdx.x;
  if (i >= per * B) return;
  const long long b = i / per;
  dy[i] = (float)(2.0 * ((double)y[i] - (double)t[i]) / ((double)B * den[b]));
}

// The BF16 value of a finite FP32 x (its upper 16 bits after round to nearest,
// ties to even), returned as the FP32 number it represents.
__device__ inline float bf16_round(float x) {
  const unsigned u = __float_as_uint(x);
  return __uint_as_float((u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u);
}

// q = the BF16 rounding of the master parameters p (the weights the network
// computes with).
__global__ __launch_bounds__(NNT) void k_quantize_bf16(const float* __restrict__ p,
                                                       float* __restrict__ q, long long n) {
  const long long i = (long long)blockIdx.x * NNT + threadIdx.x;
  if (i < n) q[i] = bf16_round(p[i]);
}

// Adam (Kingma & Ba 2015) on the FP32 master parameters p: bc1 = 1 - beta1^step,
// bc2 = 1 - beta2^step; q gets the updated parameters rounded to BF16.
__global__ __launch_bounds__(NNT) void k_adam(float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v,
                                              long long n, float lr, float beta1, float beta2,
                                              float bc1, float bc2, float eps, float* __restrict__ q) {
  const long long i = (long long)blockIdx.x * NNT + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = beta1 * m[i] + (1.0f - beta1) * gi;
  const float vi = beta2 * v[i] + (1.0f - beta2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
  p[i] = pi;
  q[i] = bf16_round(pi);
}

// ---------------------------------------------------------------------------
// Tiles of a problem: features and the blended initial guess.
// ---------------------------------------------------------------------------
// f[t] = [(Re keps / k0^2 - 1) / 4, Re b, Im b] on the n x n tile t whose
// corner is (pml_y + oy[t], pml_x + ox[t]).
__global__ __launch_bounds__(NNT) void k_nn_features(const double2* __restrict__ keps,
                                                     const double2* __restrict__ b, double k0sq,
                                                     int nx, int pml_x, int pml_y,
                                                     const int2* __restrict__ org, int n,
                                                     float* __restrict__ f) {
  const int tile = blockIdx.y;
  const long long p = (long long)blockIdx.x * NNT + threadIdx.x;
  if (p >= (long long)n * n) return;
  const int y = (int)(p / n), x = (int)(p % n);
  const int2 o = org[tile];
  const long long g = (long long)(pml_y + o.y + y) * nx + (pml_x + o.x + x);
  const long long per = (long long)n * n;
  float* ft = f + (long long)tile * 3 * per;
  ft[p] = (float)((keps[g].x / k0sq - 1.0) * 0.25);
  ft[per + p] = (float)b[g].x;
  ft[2 * per + p] = (float)b[g].y;
}

// t[tile] = [Re x, Im x] on the n x n tile (same placement as k_nn_features).
__global__ __launch_bounds__(NNT) void k_nn_fields(const double2* __restrict__ x, int nx, int pml_x,
                                                   int pml_y, const int2* __restrict__ org, int n,
                                                   float* __restrict__ t) {
  const int tile = blockIdx.y;
  const long long p = (long long)blockIdx.x * NNT + threadIdx.x;
  if (p >= (long long)n * n) return;
  const int y = (int)(p / n), xx = (int)(p % n);
  const int2 o = org[tile];
  const long long g = (long long)(pml_y + o.y + y) * nx + (pml_x + o.x + xx);
  const long long per = (long long)n * n;
  t[(long long)tile * 2 * per + p] = (float)x[g].x;
  t[(long long)tile * 2 * per + per + p] = (float)x[g].y;
}

__device__ inline double tile_w(int i, int n, bool first, bool last) {
  if ((first && i < n / 2) || (last && i >= n / 2)) return 1.0;
  const double s = sinpi((i + 0.5) / n);
  return s * s;
}

// x0 = sum_t w_t pred_t / sum_t w_t on the interior, 0 in the global PML.
// Tile origins along each axis: oy[0..nty), ox[0..ntx) (interior coordinates);
// pred[(ty * ntx + tx)] holds (2, n, n).
__global__ __launch_bounds__(NNT) void k_nn_blend(const float* __restrict__ pred,
                                                  const int* __restrict__ oy, int nty,
                                                  const int* __restrict__ ox, int ntx, int n,
                                                  int pml_x, int pml_y, int inx, int iny, int nx,
                                                  int ny, double2* __restrict__ x0) {
  const long long g = (long long)blockIdx.x * NNT + threadIdx.x;
  if (g >= (long long)nx * ny) return;
  const int gy = (int)(g / nx), gx = (int)(g % nx);
  const int iy = gy - pml_y, ix = gx - pml_x;
  double2 out = make_double2(0.0, 0.0);
  if (iy >= 0 && iy < iny && ix >= 0 && ix < inx) {
    const long long per = (long long)n * n;
    double re = 0.0, im = 0.0, ws = 0.0;
    for (int a = 0; a < nty; ++a) {
      const int ly = iy - oy[a];
      if (ly < 0 || ly >= n) continue;
      const double wy = tile_w(ly, n, a == 0, a == nty - 1);
      for (int c = 0; c < ntx; ++c) {
        const int lx = ix - ox[c];
        if (lx < 0 || lx >= n) continue;
        const double w = wy * tile_w(lx, n, c == 0, c == ntx - 1);
        const float* pt = pred + (long long)(a * ntx + c) * 2 * per;
        re += w * pt[(long long)ly * n + lx];
        im += w * pt[per + (long long)ly * n + lx];
        ws += w;
      }
    }
    if (ws > 0.0) out = make_double2(re / ws, im / ws);
  }
  x0[g] = out;
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
void nn_gemm(hipStream_t st, int batch, int M, int N, int K, const float* A, long long sAb,
             long long sAm, long long sAk, const float* B, long long sBb, long long sBk,
             long long sBn, float* C, long long sCb, long long sCm, long long sCn, float alpha,
             float beta) {
  GemmArgs g{A, B, C, M, N, K, sAb, sAm, sAk, sBb, sBk, sBn, sCb, sCm, sCn, alpha, beta};
  if (N <= 32 && K <= 256) {
    // 16-byte loads along the rows of A when every row start is 16-byte aligned
    const bool vec = sAk == 1 && sAm % 4 == 0 && sAb % 4 == 0 &&
                     (reinterpret_cast<uintptr_t>(A) & 15) == 0;
    dim3 grid((M + 63) / 64, 1, batch);
    if (vec) STF_LAUNCH((k_gemm_tall<true>), grid, dim3(256), 0, st, g);
    else STF_LAUNCH((k_gemm_tall<false>), grid, dim3(256), 0, st, g);
    return;
  }
  if (K <= 64) {
    dim3 grid((N + 63) / 64, (M + 63) / 64, batch);
    STF_LAUNCH(k_gemm_mfma, grid, dim3(256), 0, st, g);
    return;
  }
  if (N <= 32) {
    dim3 grid((N + 31) / 32, (M + 127) / 128, batch);
    STF_LAUNCH((k_gemm<128, 32>), grid, dim3(256), 0, st, g);
  } else {
    dim3 grid((N + 63) / 64, (M + 63) / 64, batch);
    STF_LAUNCH((k_gemm<64, 64>), grid, dim3(256), 0, st, g);
  }
}

void nn_dft_y(hipStream_t st, const float* T, const float2* ey, int planes, int n, int M,
              bool grad_scale, float2* H) {
  if (2 * M * M > 4 * NNT) throw Error(STF_EINVAL, "too many modes for the y transform");
  const size_t lds = (size_t)n * 2 * M * sizeof(float) + (size_t)2 * M * 64 * sizeof(float2);
  STF_LAUNCH(k_dft_y, dim3(planes), dim3(NNT), lds, st, T, ey, n, M, grad_scale ? 1 : 0, H);
}

bool nn_spec_inv_ok(int n, int M) { return n % 16 == 0 && n <= 1024 && M >= 1 && M <= 22; }
// the float4 stores of k_spec_inv: 16-byte aligned planes
bool nn_spec_inv_out_ok(const float* out, long long npix) {
  return (reinterpret_cast<uintptr_t>(out) & 15) == 0 && npix % 4 == 0;
}

void nn_spec_inv(hipStream_t st, const float2* G, const float2* ex, int planes, int n, int M,
                 bool weighted, const float* ainv, float alpha, float beta, float* out, long long npix) {
  if (!nn_spec_inv_ok(n, M) || !nn_spec_inv_out_ok(out, npix))
    throw Error(STF_EINVAL, "nn: inverse transform shape or alignment");
  const size_t lds = (size_t)4 * M * (n + 16) * sizeof(float);
  if (n == 256 && M == 16) {
    STF_LAUNCH((k_spec_inv_t<256, 16>), dim3(planes), dim3(256), lds, st, G, ex, weighted ? 1 : 0,
                       ainv, alpha, beta, out, npix);
    return;
  }
  STF_LAUNCH(k_spec_inv, dim3(planes), dim3(256), lds, st, G, ex, n, M, weighted ? 1 : 0, ainv,
                     alpha, beta, out, npix);
}

bool nn_spec_pw_ok(int n, int M, int W) { return n == 256 && M == 16 && W == 16; }

void nn_spec_rows(hipStream_t st, const float2* G, const float2* ex, int planes, int n, int M, float* S) {
  if (n != 256 || M != 16) throw Error(STF_EINVAL, "nn: x-inverse rows of the compiled shape only");
  STF_LAUNCH((k_spec_rows_t<256, 16>), dim3(planes), dim3(256), 0, st, G, ex, S);
}

void nn_spec_pw(hipStream_t st, const float* S, const float* ainv, float alpha, const float* hin,
                const float* Wm, const float* bias, long long npix, int B, int n, int M, int W, bool act,
                float* out) {
  if (!nn_spec_pw_ok(n, M, W) || npix != (long long)n * n ||
      (reinterpret_cast<uintptr_t>(hin) & 15) != 0 || (reinterpret_cast<uintptr_t>(out) & 15) != 0)
    throw Error(STF_EINVAL, "nn: fused spectral + pointwise layer shape or alignment");
  const dim3 grid(256 / 64, 256 / 16, B);
  if (act)
    STF_LAUNCH((k_spec_pw_t<256, 16, 16, true>), grid, dim3(256), 0, st, S, ainv, alpha, hin, Wm,
                       bias, npix, out);
  else
    STF_LAUNCH((k_spec_pw_t<256, 16, 16, false>), grid, dim3(256), 0, st, S, ainv, alpha, hin, Wm,
                       bias, npix, out);
}

void nn_dft_x_inv(hipStream_t st, const float2* G, const float2* ex, int planes, int n, int M,
                  bool weighted, float* S) {
  dim3 grid((2 * M * n + NNT - 1) / NNT, planes);
  STF_LAUNCH(k_dft_x_inv, grid, dim3(NNT), (size_t)2 * M * M * sizeof(float2), st, G, ex,
                     n, M, weighted ? 1 : 0, S);
}

void nn_mix_fwd(hipStream_t st, const float2* H, const float* Rre, const float* Rim, int B, int W,
                int NM, float2* G) {
  long long tot = (long long)B * W * NM;
  STF_LAUNCH(k_mix_fwd, dim3((unsigned)((tot + NNT - 1) / NNT)), dim3(NNT), 0, st, H, Rre,
                     Rim, B, W, NM, G);
}

void nn_mix_bwd(hipStream_t st, const float2* H, const float2* dG, const float* Rre,
                const float* Rim, int B, int W, int NM, float2* dH, float* dRre, float* dRim) {
  long long tot = (long long)B * W * NM;
  STF_LAUNCH(k_mix_bwd_h, dim3((unsigned)((tot + NNT - 1) / NNT)), dim3(NNT), 0, st, dG,
                     Rre, Rim, B, W, NM, dH);
  long long tr = (long long)W * W * NM;
  STF_LAUNCH(k_mix_bwd_r, dim3((unsigned)((tr + NNT - 1) / NNT)), dim3(NNT), 0, st, H, dG,
                     B, W, NM, dRre, dRim);
}

#define NN_PW_CASES(X) X(3, 16) X(16, 16) X(16, 2) X(3, 4) X(4, 4) X(4, 2) X(3, 8) X(8, 8) X(8, 2) \
  X(3, 32) X(32, 32) X(32, 2)

bool nn_width_supported(int cin, int w) {
#define NN_CASE(a, b) if (cin == a && w == b) return true;
  NN_PW_CASES(NN_CASE)
#undef NN_CASE
  return false;
}

void nn_pw_fwd(hipStream_t st, int ci, int co, bool act, const float* in, const float* Wm,
               const float* bias, const float* add, long long npix, int B, float* pre, float* out) {
  const unsigned grid = (unsigned)((npix * B + NNT - 1) / NNT);
#define NN_CASE(a, b)                                                                            \
  if (ci == a && co == b) {                                                                      \
    if (act)                                                                                     \
      STF_LAUNCH((k_pw_fwd<a, b, true>), dim3(grid), dim3(NNT), 0, st, in, Wm, bias, add, \
                         npix, B, pre, out);                                                     \
    else                                                                                         \
      STF_LAUNCH((k_pw_fwd<a, b, false>), dim3(grid), dim3(NNT), 0, st, in, Wm, bias,    \
                         add, npix, B, pre, out);                                                \
    return;                                                                                      \
  }
  NN_PW_CASES(NN_CASE)
#undef NN_CASE
  throw Error(STF_EINVAL, "unsupported channel counts of a pointwise layer");
}

int nn_pw_bwd_blocks() { return 512; }

void nn_pw_bwd(hipStream_t st, int ci, int co, bool act, const float* dout, const float* pre,
               const float* in, const float* Wm, long long npix, int B, float* dpre, float* din,
               float* partial, float* grad_w) {
  const int nblk = nn_pw_bwd_blocks();
#define NN_CASE(a, b)                                                                            \
  if (ci == a && co == b) {                                                                      \
    if (act)                                                                                     \
      STF_LAUNCH((k_pw_bwd<a, b, true>), dim3(nblk), dim3(NNT), 0, st, dout, pre, in, Wm, \
                         npix, B, dpre, din, partial);                                           \
    else                                                                                         \
      STF_LAUNCH((k_pw_bwd<a, b, false>), dim3(nblk), dim3(NNT), 0, st, dout, pre, in,   \
                         Wm, npix, B, dpre, din, partial);                                       \
    const int cnt = a * b + b;                                                                   \
    STF_LAUNCH(k_sum_partials, dim3((cnt + NNT - 1) / NNT), dim3(NNT), 0, st, partial,   \
                       nblk, cnt, cnt, grad_w);                                                  \
    return;                                                                                      \
  }
  NN_PW_CASES(NN_CASE)
#undef NN_CASE
  throw Error(STF_EINVAL, "unsupported channel counts of a pointwise layer");
}

int nn_loss_blocks() { return 64; }

void nn_loss(hipStream_t st, const float* y, const float* t, long long per, int B, double* partial,
             double* den, double* loss, float* dy) {
  const int nblk = nn_loss_blocks();
  STF_LAUNCH(k_loss_partial, dim3(nblk, B), dim3(NNT), 0, st, y, t, per, nblk, partial);
  STF_LAUNCH(k_loss_final, dim3(1), dim3(64), 0, st, partial, B, nblk, den, loss);
  if (dy)
    STF_LAUNCH(k_loss_grad, dim3((unsigned)((per * B + NNT - 1) / NNT)), dim3(NNT), 0, st, y,
                       t, den, per, B, dy);
}

void nn_adam(hipStream_t st, float* p, const float* g, float* m, float* v, long long n, double lr,
             int step, double beta1, double beta2, double eps, float* q) {
  const float bc1 = (float)(1.0 - std::pow(beta1, step));
  const float bc2 = (float)(1.0 - std::pow(beta2, step));
  STF_LAUNCH(k_adam, dim3((unsigned)((n + NNT - 1) / NNT)), dim3(NNT), 0, st, p, g, m, v, n,
                     (float)lr, (float)beta1, (float)beta2, bc1, bc2, (float)eps, q);
}

void nn_quantize_bf16(hipStream_t st, const float* p, float* q, long long n) {
  STF_LAUNCH(k_quantize_bf16, dim3((unsigned)((n + NNT - 1) / NNT)), dim3(NNT), 0, st, p, q, n);
}

void nn_features(hipStream_t st, const double2* keps, const double2* b, double k0sq, int nx,
                 int pml_x, int pml_y, const int2* org, int ntiles, int n, float* f) {
  dim3 grid((unsigned)(((long long)n * n + NNT - 1) / NNT), ntiles);
  STF_LAUNCH(k_nn_features, grid, dim3(NNT), 0, st, keps, b, k0sq, nx, pml_x, pml_y, org, n,
                     f);
}

void nn_fields(hipStream_t st, const double2* x, int nx, int pml_x, int pml_y, const int2* org,
               int ntiles, int n, float* t) {
  dim3 grid((unsigned)(((long long)n * n + NNT - 1) / NNT), ntiles);
  STF_LAUNCH(k_nn_fields, grid, dim3(NNT), 0, st, x, nx, pml_x, pml_y, org, n, t);
}

void nn_blend(hipStream_t st, const float* pred, const int* oy, int nty, const int* ox, int ntx,
              int n, int pml_x, int pml_y, int inx, int iny, int nx, int ny, double2* x0) {
  const long long N = (long long)nx * ny;
  STF_LAUNCH(k_nn_blend, dim3((unsigned)((N + NNT - 1) / NNT)), dim3(NNT), 0, st, pred, oy,
                     nty, ox, ntx, n, pml_x, pml_y, inx, iny, nx, ny, x0);
}

}  // namespace stf
