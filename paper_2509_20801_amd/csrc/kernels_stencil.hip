// Global FP64 operator kernels: node permittivity (Eq. (3)) and the five-point
// SC-PML stencil (Eqs. (2) and (9)), plus reductions.
//
// Layout: node arrays row-major [ny][nx] of double2 (complex128), x fastest.
// The operator is stored implicitly: keps[n] = k0^2 eps_bar(n) per node and four
// 1D coupling arrays (x: w, e per column; y: w, e per row), so one apply reads
// x (16 B) + keps (16 B) and writes y (16 B) per node; the five x reads of a
// node's stencil come from cache.  Blocks are 64 x 4 nodes so a wavefront reads
// one contiguous 1 KiB row segment.
#include "cplx.h"
#include "stf_internal.h"

namespace stf {

namespace {

constexpr int SBX = 64, SBY = 4;

__global__ __launch_bounds__(256) void k_node_keps(const double2* __restrict__ cells,
                                                   double2* __restrict__ keps, int nx, int ny,
                                                   double k0sq) {
  int i = blockIdx.x * SBX + threadIdx.x;
  int j = blockIdx.y * SBY + threadIdx.y;
  if (i >= nx || j >= ny) return;
  long long w = nx + 1;
  // Node (i, j) touches cells (i, j), (i+1, j), (i, j+1), (i+1, j+1).
  double2 a = cells[(long long)j * w + i], b = cells[(long long)j * w + i + 1];
  double2 c = cells[(long long)(j + 1) * w + i], d = cells[(long long)(j + 1) * w + i + 1];
  double2 s = make_double2(0.25 * ((a.x + b.x) + (c.x + d.x)), 0.25 * ((a.y + b.y) + (c.y + d.y)));
  keps[(long long)j * nx + i] = make_double2(k0sq * s.x, k0sq * s.y);
}

template <int MODE>
__global__ __launch_bounds__(256) void k_stencil(const double2* __restrict__ x,
                                                 const double2* __restrict__ b,
                                                 double2* __restrict__ y,
                                                 const double2* __restrict__ keps,
                                                 const double2* __restrict__ cxw,
                                                 const double2* __restrict__ cxe,
                                                 const double2* __restrict__ cyw,
                                                 const double2* __restrict__ cye, int nx, int ny,
                                                 double* __restrict__ partial) {
  int i = blockIdx.x * SBX + threadIdx.x;
  int j = blockIdx.y * SBY + threadIdx.y;
  double loc = 0.0;
  if (i < nx && j < ny) {
    long long n = (long long)j * nx + i;
    double2 aw = cxw[i], ae = cxe[i], as = cyw[j], an = cye[j];
    double2 ke = keps[n];
    // Diagonal: k0^2 eps_bar minus all four couplings (Dirichlet neighbours included).
    double2 dg = make_double2(ke.x - ((aw.x + ae.x) + (as.x + an.x)),
                              ke.y - ((aw.y + ae.y) + (as.y + an.y)));
    double2 acc = cmul(dg, x[n]);
    if (i > 0) acc = cfma(aw, x[n - 1], acc);
    if (i < nx - 1) acc = cfma(ae, x[n + 1], acc);
    if (j > 0) acc = cfma(as, x[n - nx], acc);
    if (j < ny - 1) acc = cfma(an, x[n + nx], acc);
    if (MODE == 0) {
      y[n] = acc;
    } else {
      double2 r = csub(b[n], acc);
      y[n] = r;
      loc = r.x * r.x + r.y * r.y;
    }
  }
  if (MODE == 1) {
    __shared__ double red[4];
    int tid = threadIdx.y * SBX + threadIdx.x;
    double s = wave_sum(loc);
    if ((tid & 63) == 0) red[tid >> 6] = s;
    __syncthreads();
    if (tid == 0) partial[blockIdx.y * gridDim.x + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
  }
}

// y_s = A x_s for NR vectors (blockIdx.z-free: every thread applies its
// node's coefficients, loaded once, to all of them; the arithmetic per vector
// is that of k_stencil<0>).
template <int NR>
__global__ __launch_bounds__(256) void k_stencil_set(StencilSet S, const double2* __restrict__ keps,
                                                     const double2* __restrict__ cxw,
                                                     const double2* __restrict__ cxe,
                                                     const double2* __restrict__ cyw,
                                                     const double2* __restrict__ cye, int nx, int ny) {
  int i = blockIdx.x * SBX + threadIdx.x;
  int j = blockIdx.y * SBY + threadIdx.y;
  if (i >= nx || j >= ny) return;
  long long n = (long long)j * nx + i;
  double2 aw = cxw[i], ae = cxe[i], as = cyw[j], an = cye[j];
  double2 ke = keps[n];
  double2 dg = make_double2(ke.x - ((aw.x + ae.x) + (as.x + an.x)),
                            ke.y - ((aw.y + ae.y) + (as.y + an.y)));
#pragma unroll
  for (int s = 0; s < NR; ++s) {
    const double2* __restrict__ x = S.x[s];
    double2 acc = cmul(dg, x[n]);
    if (i > 0) acc = cfma(aw, x[n - 1], acc);
    if (i < nx - 1) acc = cfma(ae, x[n + 1], acc);
    if (j > 0) acc = cfma(as, x[n - nx], acc);
    if (j < ny - 1) acc = cfma(an, x[n + nx], acc);
    S.y[s][n] = acc;
  }
}

// r_s = b_s - A x_s for NR right-hand sides with per-block partial |r_s|^2,
// each node's coefficients loaded once (per vector the arithmetic and the
// block sums of k_stencil<1>).
template <int NR>
__global__ __launch_bounds__(256) void k_residual_set(ResidualSet S, const double2* __restrict__ keps,
                                                      const double2* __restrict__ cxw,
                                                      const double2* __restrict__ cxe,
                                                      const double2* __restrict__ cyw,
                                                      const double2* __restrict__ cye, int nx, int ny) {
  int i = blockIdx.x * SBX + threadIdx.x;
  int j = blockIdx.y * SBY + threadIdx.y;
  double loc[NR];
#pragma unroll
  for (int s = 0; s < NR; ++s) loc[s] = 0.0;
  if (i < nx && j < ny) {
    long long n = (long long)j * nx + i;
    double2 aw = cxw[i], ae = cxe[i], as = cyw[j], an = cye[j];
    double2 ke = keps[n];
    double2 dg = make_double2(ke.x - ((aw.x + ae.x) + (as.x + an.x)),
                              ke.y - ((aw.y + ae.y) + (as.y + an.y)));
#pragma unroll
    for (int s = 0; s < NR; ++s) {
      const double2* __restrict__ x = S.x[s];
      double2 acc = cmul(dg, x[n]);
      if (i > 0) acc = cfma(aw, x[n - 1], acc);
      if (i < nx - 1) acc = cfma(ae, x[n + 1], acc);
      if (j > 0) acc = cfma(as, x[n - nx], acc);
      if (j < ny - 1) acc = cfma(an, x[n + nx], acc);
      double2 r = csub(S.b[s][n], acc);
      S.r[s][n] = r;
      loc[s] = r.x * r.x + r.y * r.y;
    }
  }
  __shared__ double red[NR][4];
  int tid = threadIdx.y * SBX + threadIdx.x;
#pragma unroll
  for (int s = 0; s < NR; ++s) {
    double v = wave_sum(loc[s]);
    if ((tid & 63) == 0) red[s][tid >> 6] = v;
  }
  __syncthreads();
  if (tid < NR)
    S.partial[tid][blockIdx.y * gridDim.x + blockIdx.x] = (red[tid][0] + red[tid][1]) + (red[tid][2] + red[tid][3]);
}

// out_s[0] = the sum of the n partials of right-hand side s (blockIdx.x = s),
// also written to host_out_s[0] when given (device-visible host memory).
__global__ __launch_bounds__(256) void k_reduce_sum_set(ResidualSet S, int n) {
  __shared__ double red[4];
  const int sy = blockIdx.x;
  const double* __restrict__ partial = S.partial[sy];
  double s = 0.0;
  for (int t = threadIdx.x; t < n; t += 256) s += partial[t];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double v = (red[0] + red[1]) + (red[2] + red[3]);
    S.out[sy][0] = v;
    if (S.host_out[sy]) S.host_out[sy][0] = v;
  }
}

__global__ __launch_bounds__(256) void k_reduce_sum(const double* __restrict__ partial, int n,
                                                    double* __restrict__ out) {
  __shared__ double red[4];
  double s = 0.0;
  for (int t = threadIdx.x; t < n; t += 256) s += partial[t];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[0] = (red[0] + red[1]) + (red[2] + red[3]);
}

// Power through a grid line (the line integral of Re(E x H*) / 2, Sec. 3.2):
// the line lies between node rows j0 and j0 + 1 (constant y; nodes x in
// [lo, hi): element t at (j0, lo + t) and (j0 + 1, lo + t), so stride_t = 1 and
// stride_n = nx) or between node columns (stride_t = nx, stride_n = 1).  With
// H_x = (j / k0) dE/dy (or -H_y = (j / k0) dE/dx) on the line, each element adds
// Re(e_mid conj(j (b - a) / (k0 d))) = Im(e_mid conj(b - a)) / (k0 d); one
// workgroup sums in a fixed order and scales by dl / 2.
__global__ __launch_bounds__(256) void k_line_flux(const double2* __restrict__ e, long long base,
                                                   long long stride_t, long long stride_n, int count,
                                                   double inv_k0d, double half_dl,
                                                   double* __restrict__ out) {
  __shared__ double red[4];
  double s = 0.0;
  for (int t = threadIdx.x; t < count; t += 256) {
    const long long n = base + (long long)t * stride_t;
    const double2 a = e[n], b = e[n + stride_n];
    const double mx = 0.5 * (a.x + b.x), my = 0.5 * (a.y + b.y);   // mean across the line
    const double rx = b.x - a.x, ry = b.y - a.y;                    // difference across it
    s += (my * rx - mx * ry) * inv_k0d;           // Im(mean conj(difference)) / (k0 d)
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[0] = ((red[0] + red[1]) + (red[2] + red[3])) * half_dl;
}

// Near-to-far-field transform (the RCS of Sec. 3.1): per angle (block),
// F(phi) = sum over the contour elements of [du/dn - j k0 (rhat . n) u] exp(j k0 rhat . r) dl
// on the rectangle through the half-node lines x = (i0 + 1/2) dx, (i1 + 1/2) dx,
// y = (j0 + 1/2) dy, (j1 + 1/2) dy: u is the mean of the two node lines an edge
// separates, du/dn their difference over the step times the outward sign; the
// elements are the nodes strictly inside each edge's span.  A fixed-order
// block reduction writes F[blockIdx.x].
__global__ __launch_bounds__(256) void k_far_field(const double2* __restrict__ e, int nx, int i0,
                                                   int i1, int j0, int j1, double dx, double dy,
                                                   double k0, const double* __restrict__ phis,
                                                   double2* __restrict__ F) {
  __shared__ double red[2][4];
  const double phi = phis[blockIdx.x];
  const double c = cos(phi), s = sin(phi);
  const int nh = i1 - i0, nv = j1 - j0;               // elements per horizontal / vertical edge
  const int total = 2 * nh + 2 * nv;
  double ar = 0.0, ai = 0.0;
  for (int t = threadIdx.x; t < total; t += 256) {
    long long na, nb;                                  // the two node lines' nodes
    double xe, ye, nrm, dl, inv, rn;
    if (t < 2 * nh) {                                  // bottom (t < nh) or top edge
      const int top = t >= nh, i = i0 + 1 + (top ? t - nh : t);
      const int row = top ? j1 : j0;
      na = (long long)row * nx + i;
      nb = na + nx;
      xe = i * dx;
      ye = (row + 0.5) * dy;
      nrm = top ? 1.0 : -1.0;
      dl = dx;
      inv = 1.0 / dy;
      rn = s * nrm;
    } else {                                           // left or right edge
      const int u = t - 2 * nh, right = u >= nv, j = j0 + 1 + (right ? u - nv : u);
      const int col = right ? i1 : i0;
      na = (long long)j * nx + col;
      nb = na + 1;
      xe = (col + 0.5) * dx;
      ye = j * dy;
      nrm = right ? 1.0 : -1.0;
      dl = dy;
      inv = 1.0 / dx;
      rn = c * nrm;
    }
    const double2 a = e[na], b = e[nb];
    const double2 um = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y + b.y));
    const double2 dn = make_double2((b.x - a.x) * inv * nrm, (b.y - a.y) * inv * nrm);
    // g = dn - j k0 rn um
    const double2 g = make_double2(dn.x + k0 * rn * um.y, dn.y - k0 * rn * um.x);
    double sp, cp;
    sincos(k0 * (c * xe + s * ye), &sp, &cp);
    ar += (g.x * cp - g.y * sp) * dl;
    ai += (g.x * sp + g.y * cp) * dl;
  }
  ar = wave_sum(ar);
  ai = wave_sum(ai);
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = ar;
    red[1][threadIdx.x >> 6] = ai;
  }
  __syncthreads();
  if (threadIdx.x == 0)
    F[blockIdx.x] = make_double2((red[0][0] + red[0][1]) + (red[0][2] + red[0][3]),
                                 (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]));
}

__global__ __launch_bounds__(256) void k_check_finite(const double* __restrict__ a, long long n,
                                                      int* __restrict__ flag) {
  long long t = (long long)blockIdx.x * 256 + threadIdx.x;
  int bad = 0;
  for (; t < n; t += (long long)gridDim.x * 256) bad |= !isfinite(a[t]);
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

}  // namespace

void launch_node_keps(hipStream_t st, const double2* cells, double2* keps, int nx, int ny,
                      double k0sq) {
  dim3 blk(SBX, SBY), grd((nx + SBX - 1) / SBX, (ny + SBY - 1) / SBY);
  STF_LAUNCH(k_node_keps, grd, blk, 0, st, cells, keps, nx, ny, k0sq);
}

int stencil_partial_blocks(int nx, int ny) {
  return ((nx + SBX - 1) / SBX) * ((ny + SBY - 1) / SBY);
}

void launch_stencil_set(hipStream_t st, int nr, const StencilSet& S, const double2* keps,
                        const double2* cxw, const double2* cxe, const double2* cyw,
                        const double2* cye, int nx, int ny) {
  STF_REQUIRE(nr >= 1 && nr <= MAX_RHS, "1 to 4 vectors per stencil launch");
  dim3 blk(SBX, SBY), grd((nx + SBX - 1) / SBX, (ny + SBY - 1) / SBY);
#define STF_CALL(NR) \
  STF_LAUNCH((k_stencil_set<NR>), grd, blk, 0, st, S, keps, cxw, cxe, cyw, cye, nx, ny)
  if (nr == 1) STF_CALL(1);
  else if (nr == 2) STF_CALL(2);
  else if (nr == 3) STF_CALL(3);
  else STF_CALL(4);
#undef STF_CALL
}

void launch_stencil(hipStream_t st, int mode, const double2* x, const double2* b, double2* y,
                    const double2* keps, const double2* cxw, const double2* cxe,
                    const double2* cyw, const double2* cye, int nx, int ny, double* partial,
                    int* nblocks_out) {
  dim3 blk(SBX, SBY), grd((nx + SBX - 1) / SBX, (ny + SBY - 1) / SBY);
  if (mode == 0)
    STF_LAUNCH(k_stencil<0>, grd, blk, 0, st, x, b, y, keps, cxw, cxe, cyw, cye, nx, ny,
                       partial);
  else
    STF_LAUNCH(k_stencil<1>, grd, blk, 0, st, x, b, y, keps, cxw, cxe, cyw, cye, nx, ny,
                       partial);
  if (nblocks_out) *nblocks_out = grd.x * grd.y;
}

void launch_line_flux(hipStream_t st, const double2* e, int nx, int axis, int index, int lo, int hi,
                      double k0, double dx, double dy, double* out) {
  const long long base = axis == 1 ? (long long)index * nx + lo : (long long)lo * nx + index;
  const long long st_t = axis == 1 ? 1 : nx, st_n = axis == 1 ? nx : 1;
  const double d = axis == 1 ? dy : dx, dl = axis == 1 ? dx : dy;
  STF_LAUNCH(k_line_flux, dim3(1), dim3(256), 0, st, e, base, st_t, st_n, hi - lo,
                     1.0 / (k0 * d), 0.5 * dl, out);
}

void launch_far_field(hipStream_t st, const double2* e, int nx, int i0, int i1, int j0, int j1,
                      double dx, double dy, double k0, const double* phis, int nang, double2* F) {
  STF_LAUNCH(k_far_field, dim3(nang), dim3(256), 0, st, e, nx, i0, i1, j0, j1, dx, dy, k0,
                     phis, F);
}

void launch_residual_set(hipStream_t st, int nr, const ResidualSet& S, const double2* keps,
                         const double2* cxw, const double2* cxe, const double2* cyw,
                         const double2* cye, int nx, int ny) {
  STF_REQUIRE(nr >= 1 && nr <= MAX_RHS, "1 to 4 vectors per residual launch");
  dim3 blk(SBX, SBY), grd((nx + SBX - 1) / SBX, (ny + SBY - 1) / SBY);
#define STF_CALL(NR) \
  STF_LAUNCH((k_residual_set<NR>), grd, blk, 0, st, S, keps, cxw, cxe, cyw, cye, nx, ny)
  if (nr == 1) STF_CALL(1);
  else if (nr == 2) STF_CALL(2);
  else if (nr == 3) STF_CALL(3);
  else STF_CALL(4);
#undef STF_CALL
  STF_LAUNCH(k_reduce_sum_set, dim3(nr), dim3(256), 0, st, S, (int)(grd.x * grd.y));
}

void launch_reduce_sum(hipStream_t st, const double* partial, int n, double* out) {
  STF_LAUNCH(k_reduce_sum, dim3(1), dim3(256), 0, st, partial, n, out);
}

void launch_check_finite(hipStream_t st, const double* a, long long n, int* flag) {
  long long g = (n + 255) / 256;
  if (g > 2048) g = 2048;
  if (g < 1) g = 1;
  STF_LAUNCH(k_check_finite, dim3((unsigned)g), dim3(256), 0, st, a, n, flag);
}

}  // namespace stf
