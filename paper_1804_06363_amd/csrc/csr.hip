// Passes of RBCG / RBI over a general sparse affine problem (eq. 12, Sec. 2.3):
// A(theta) = sum_q theta_q A_q with every term stored on one shared pattern.
//
// Layout (StencilGeom with csr != 0): rows in storage (colour-major) order, grouped in
// slices of 64 rows; entry k of row 64 s + l sits at sptr[s] + 64 k + l, so the 64 lanes
// of a wavefront read consecutive words.  Off-diagonal entries only (the diagonal is kept
// apart); padding entries point at their own row with value 0 and are skipped.  For each query the
// coefficient table holds theta (Q doubles).
//
// Every kernel runs on (query group) x (chunk of 1024 rows) blocks, 4 rows per thread;
// partial sums go to part[b][chunk] like the stencil passes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "internal.h"
#include "kernels.h"

namespace rb {

constexpr int kCsrThreads = 256;
constexpr int kCsrRows = 4;  // rows per thread

int csr_chunks(int rows) {
  return (rows + kCsrThreads * kCsrRows - 1) / (kCsrThreads * kCsrRows);
}

// theta of queries q0..q0+QPB-1 into LDS; returns the mask of live queries
template <int QPB>
__device__ __forceinline__ unsigned csr_group(const StencilGeom& g, const double* coef, int q0,
                                              int B, const int* active, double* sh) {
  unsigned mask = 0;
#pragma unroll
  for (int k = 0; k < QPB; ++k) {
    const int b = q0 + k;
    if (b < B && (!active || active[b])) mask |= 1u << k;
  }
  if (mask)
    for (int e = threadIdx.x; e < QPB * g.ct_size; e += blockDim.x) {
      const int k = e / g.ct_size;
      sh[e] = (q0 + k < B) ? coef[(size_t)(q0 + k) * g.ct_size + (e - k * g.ct_size)] : 0.0;
    }
  __syncthreads();
  return mask;
}

template <int QPB>
__device__ __forceinline__ void csr_partials(const double (&acc)[QPB], unsigned mask, int q0,
                                             int chunk, int chunks, double* part,
                                             double* red /* 4*QPB */) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < QPB; ++k) {
    const double v = rbk::wave_sum(acc[k]);
    if (lane == 0) red[k * 4 + w] = v;
  }
  __syncthreads();
  if (threadIdx.x < QPB && ((mask >> threadIdx.x) & 1u)) {
    const int k = threadIdx.x;
    part[(size_t)(q0 + k) * chunks + chunk] =
        (red[k * 4 + 0] + red[k * 4 + 1]) + (red[k * 4 + 2] + red[k * 4 + 3]);
  }
}

// Row `row` for every live query k: d[k] = A(theta_k)_{row,row},
// off[k] = sum_{j != row} A(theta_k)_{row,j} V(k, j).  Arithmetic in T.
template <int QPB, typename T, typename V>
__device__ __forceinline__ void csr_row(const StencilGeom& g, int row, const double* th,
                                        V val, T (&d)[QPB], T (&off)[QPB]) {
  const int s = row >> 6, lane = row & 63;
  const int64_t b0 = g.sptr[s];
  const int w = (int)((g.sptr[s + 1] - b0) >> 6);
#pragma unroll
  for (int k = 0; k < QPB; ++k) {
    d[k] = T(0);
    off[k] = T(0);
  }
  for (int q = 0; q < g.Q; ++q) {
    const double dq = g.diag[(size_t)q * g.N + row];
#pragma unroll
    for (int k = 0; k < QPB; ++k) d[k] += (T)(th[k * g.ct_size + q] * dq);
  }
  for (int e = 0; e < w; ++e) {
    const int64_t at = b0 + (int64_t)e * 64 + lane;
    const int c = g.scol[at];
    double a[QPB];
#pragma unroll
    for (int k = 0; k < QPB; ++k) a[k] = 0.0;
    for (int q = 0; q < g.Q; ++q) {
      const double v = g.sval[(size_t)q * g.sval_ld + at];
#pragma unroll
      for (int k = 0; k < QPB; ++k) a[k] += th[k * g.ct_size + q] * v;
    }
    // padding entries point at the row itself with value 0; select rather than multiply,
    // since a Gauss-Seidel sweep reads its own rows before writing them (stale memory,
    // possibly not finite)
#pragma unroll
    for (int k = 0; k < QPB; ++k) {
      const T t = (T)a[k] * val(k, c);
      off[k] += c == row ? T(0) : t;
    }
  }
}

// |A(theta_k)| row sums against V >= 0: d[k] = |A_{row,row}|, off[k] = sum_{j != row}
// |A_{row,j}| V(k, j)
template <int QPB, typename V>
__device__ __forceinline__ void csr_row_abs(const StencilGeom& g, int row, const double* th,
                                            V val, double (&d)[QPB], double (&off)[QPB]) {
  const int s = row >> 6, lane = row & 63;
  const int64_t b0 = g.sptr[s];
  const int w = (int)((g.sptr[s + 1] - b0) >> 6);
#pragma unroll
  for (int k = 0; k < QPB; ++k) d[k] = off[k] = 0.0;
  for (int q = 0; q < g.Q; ++q) {
    const double dq = g.diag[(size_t)q * g.N + row];
#pragma unroll
    for (int k = 0; k < QPB; ++k) d[k] += th[k * g.ct_size + q] * dq;
  }
#pragma unroll
  for (int k = 0; k < QPB; ++k) d[k] = fabs(d[k]);
  for (int e = 0; e < w; ++e) {
    const int64_t at = b0 + (int64_t)e * 64 + lane;
    const int c = g.scol[at];
    double a[QPB];
#pragma unroll
    for (int k = 0; k < QPB; ++k) a[k] = 0.0;
    for (int q = 0; q < g.Q; ++q) {
      const double v = g.sval[(size_t)q * g.sval_ld + at];
#pragma unroll
      for (int k = 0; k < QPB; ++k) a[k] += th[k * g.ct_size + q] * v;
    }
#pragma unroll
    for (int k = 0; k < QPB; ++k) {
      const double t = fabs(a[k]) * val(k, c);
      off[k] += c == row ? 0.0 : t;
    }
  }
}

struct CsrTile {
  int chunk, q0;
};
__device__ __forceinline__ CsrTile csr_tile(int chunks, int qpb) {
  return CsrTile{(int)(blockIdx.x % chunks), (int)(blockIdx.x / chunks) * qpb};
}

// ---- y = A u (mode 0) or y = rhs_scale rhs - A u with partial ||y||^2 (mode 1) --------
template <int QPB>
__global__ __launch_bounds__(kCsrThreads) void k_csr_apply(StencilGeom g, int64_t ld, int B,
                                                           int chunks, const double* coef,
                                                           const double* __restrict__ u,
                                                           double* __restrict__ y, int mode,
                                                           const double* __restrict__ rhs,
                                                           int64_t rhs_ld,
                                                           const double* __restrict__ rhs_scale,
                                                           const int* __restrict__ flag,
                                                           double* __restrict__ part,
                                                           double* __restrict__ part2) {
  extern __shared__ double th[];
  __shared__ double red[4 * QPB];
  const CsrTile tl = csr_tile(chunks, QPB);
  const unsigned mask = csr_group<QPB>(g, coef, tl.q0, B, mode == 1 ? flag : nullptr, th);
  if (!mask) return;
  double acc[QPB], acc2[QPB];
#pragma unroll
  for (int k = 0; k < QPB; ++k) acc[k] = acc2[k] = 0.0;
  for (int t = 0; t < kCsrRows; ++t) {
    const int row = tl.chunk * kCsrThreads * kCsrRows + t * kCsrThreads + (int)threadIdx.x;
    if (row >= g.N) continue;
    double d[QPB], off[QPB];
    csr_row<QPB, double>(g, row, th,
                         [&](int k, int c) { return u[(size_t)min(tl.q0 + k, B - 1) * ld + c]; },
                         d, off);
#pragma unroll
    for (int k = 0; k < QPB; ++k) {
      if (!((mask >> k) & 1u)) continue;
      const size_t o = (size_t)(tl.q0 + k) * ld + row;
      const double Au = d[k] * u[o] + off[k];
      if (mode == 0) {
        y[o] = Au;
      } else {
        const double r = rhs_scale[tl.q0 + k] * rhs[(size_t)(tl.q0 + k) * rhs_ld + row] - Au;
        y[o] = r;
        acc[k] += r * r;
      }
    }
    if (mode == 1 && part2) {  // (|A| |u|)_row for the rounding level of the residual
      double ad[QPB], aoff[QPB];
      csr_row_abs<QPB>(g, row, th, [&](int k, int c) {
        return fabs(u[(size_t)min(tl.q0 + k, B - 1) * ld + c]); }, ad, aoff);
#pragma unroll
      for (int k = 0; k < QPB; ++k) {
        const double a = ad[k] * fabs(u[(size_t)min(tl.q0 + k, B - 1) * ld + row]) + aoff[k];
        acc2[k] += a * a;
      }
    }
  }
  if (mode == 1) csr_partials<QPB>(acc, mask, tl.q0, tl.chunk, chunks, part, red);
  if (mode == 1 && part2) {
    __syncthreads();
    csr_partials<QPB>(acc2, mask, tl.q0, tl.chunk, chunks, part2, red);
  }
}

// ---- pass A: p_new = y + beta p_old; partial p_new^T A p_new ------------------------------
template <int QPB, typename TY>
__global__ __launch_bounds__(kCsrThreads) void k_csr_pass_a(StencilGeom g, int64_t ld, int B,
                                                            int chunks, const double* coef,
                                                            const TY* __restrict__ y,
                                                            int64_t y_ld,
                                                            const double* __restrict__ p_old,
                                                            double* __restrict__ p_new,
                                                            const double* __restrict__ beta,
                                                            const int* __restrict__ active,
                                                            double* __restrict__ part) {
  extern __shared__ double th[];
  __shared__ double red[4 * QPB];
  const CsrTile tl = csr_tile(chunks, QPB);
  const unsigned mask = csr_group<QPB>(g, coef, tl.q0, B, active, th);
  if (!mask) return;
  double acc[QPB], be[QPB];
#pragma unroll
  for (int k = 0; k < QPB; ++k) {
    acc[k] = 0.0;
    be[k] = ((mask >> k) & 1u) ? beta[tl.q0 + k] : 0.0;
  }
  auto v = [&](int k, int c) {
    const int b = min(tl.q0 + k, B - 1);
    return (double)y[(size_t)b * y_ld + c] + be[k] * p_old[(size_t)b * ld + c];
  };
  for (int t = 0; t < kCsrRows; ++t) {
    const int row = tl.chunk * kCsrThreads * kCsrRows + t * kCsrThreads + (int)threadIdx.x;
    if (row >= g.N) continue;
    double d[QPB], off[QPB];
    csr_row<QPB, double>(g, row, th, v, d, off);
#pragma unroll
    for (int k = 0; k < QPB; ++k) {
      if (!((mask >> k) & 1u)) continue;
      const double pp = v(k, row);
      p_new[(size_t)(tl.q0 + k) * ld + row] = pp;
      acc[k] += pp * (d[k] * pp + off[k]);
    }
  }
  csr_partials<QPB>(acc, mask, tl.q0, tl.chunk, chunks, part, red);
}

// ---- pass B: x += alpha p; r_out = r_in - alpha A p; partial ||r_out||^2 --------------------
template <int QPB>
__global__ __launch_bounds__(kCsrThreads) void k_csr_pass_b(StencilGeom g, int64_t ld, int B,
                                                            int chunks, const double* coef,
                                                            const double* __restrict__ p,
                                                            double* __restrict__ x,
                                                            const double* r_in, double* r_out,
                                                            const double* __restrict__ alpha,
                                                            const int* __restrict__ active,
                                                            double* __restrict__ part) {
  extern __shared__ double th[];
  __shared__ double red[4 * QPB];
  const CsrTile tl = csr_tile(chunks, QPB);
  const unsigned mask = csr_group<QPB>(g, coef, tl.q0, B, active, th);
  if (!mask) return;
  double acc[QPB], al[QPB];
#pragma unroll
  for (int k = 0; k < QPB; ++k) {
    acc[k] = 0.0;
    al[k] = ((mask >> k) & 1u) ? alpha[tl.q0 + k] : 0.0;
  }
  auto v = [&](int k, int c) { return p[(size_t)min(tl.q0 + k, B - 1) * ld + c]; };
  for (int t = 0; t < kCsrRows; ++t) {
    const int row = tl.chunk * kCsrThreads * kCsrRows + t * kCsrThreads + (int)threadIdx.x;
    if (row >= g.N) continue;
    double d[QPB], off[QPB];
    csr_row<QPB, double>(g, row, th, v, d, off);
#pragma unroll
    for (int k = 0; k < QPB; ++k) {
      if (!((mask >> k) & 1u)) continue;
      const size_t o = (size_t)(tl.q0 + k) * ld + row;
      const double pp = p[o];
      const double Ap = d[k] * pp + off[k];
      x[o] += al[k] * pp;
      const double r = r_in[o] - al[k] * Ap;
      r_out[o] = r;
      acc[k] += r * r;
    }
  }
  csr_partials<QPB>(acc, mask, tl.q0, tl.chunk, chunks, part, red);
}

// ---- Gauss-Seidel on the rows of one colour class ----------------------------------------
// y_i = (rhs_i - sum_{j != i} A_ij y_j) / A_ii with rhs_b = rhs_scale[b] rhs[b]; partial
// sums y_i rhs_i (part0) and y_i rhs2_i (part1) over the updated rows.  Arithmetic in TY.
template <int QPB, typename TY>
__global__ __launch_bounds__(kCsrThreads) void k_csr_gs(StencilGeom g, int color, int B,
                                                        int chunks, const double* coef,
                                                        TY* __restrict__ y, int64_t y_ld,
                                                        const double* __restrict__ rhs,
                                                        int64_t rhs_ld,
                                                        const double* __restrict__ rhs_scale,
                                                        const double* __restrict__ rhs2,
                                                        int64_t rhs2_ld,
                                                        const int* __restrict__ active,
                                                        double* __restrict__ part0,
                                                        double* __restrict__ part1) {
  extern __shared__ double th[];
  __shared__ double red[4 * QPB];
  const CsrTile tl = csr_tile(chunks, QPB);
  const unsigned mask = csr_group<QPB>(g, coef, tl.q0, B, active, th);
  if (!mask) return;
  const int lo = g.coff[color], hi = g.coff[color + 1];
  double a0[QPB], a1[QPB], fsc[QPB];
#pragma unroll
  for (int k = 0; k < QPB; ++k) {
    a0[k] = a1[k] = 0.0;
    fsc[k] = (rhs_scale && ((mask >> k) & 1u)) ? rhs_scale[tl.q0 + k] : 1.0;
  }
  auto v = [&](int k, int c) { return y[(size_t)min(tl.q0 + k, B - 1) * y_ld + c]; };
  for (int t = 0; t < kCsrRows; ++t) {
    const int row = lo + tl.chunk * kCsrThreads * kCsrRows + t * kCsrThreads + (int)threadIdx.x;
    if (row >= hi) continue;
    TY d[QPB], off[QPB];
    csr_row<QPB, TY>(g, row, th, v, d, off);
#pragma unroll
    for (int k = 0; k < QPB; ++k) {
      if (!((mask >> k) & 1u)) continue;
      const double fp = fsc[k] * rhs[(size_t)(tl.q0 + k) * rhs_ld + row];
      const TY nv = (TY)(((TY)fp - off[k]) / d[k]);
      y[(size_t)(tl.q0 + k) * y_ld + row] = nv;
      a0[k] += (double)nv * fp;
      if (rhs2) a1[k] += (double)nv * rhs2[(size_t)(tl.q0 + k) * rhs2_ld + row];
    }
  }
  if (part0) csr_partials<QPB>(a0, mask, tl.q0, tl.chunk, chunks, part0, red);
  if (part1) {
    __syncthreads();
    csr_partials<QPB>(a1, mask, tl.q0, tl.chunk, chunks, part1, red);
  }
}

// ---- damped Jacobi: y = z + omega D^-1 (rhs - A z), partial y^T rhs (and y^T rhs2) ---------
template <int QPB, typename TY>
__global__ __launch_bounds__(kCsrThreads) void k_csr_jacobi(StencilGeom g, int B, int chunks,
                                                            const double* coef,
                                                            const TY* __restrict__ z,
                                                            TY* __restrict__ y, int64_t y_ld,
                                                            double omega,
                                                            const double* __restrict__ rhs,
                                                            int64_t rhs_ld,
                                                            const double* __restrict__ rhs2,
                                                            int64_t rhs2_ld,
                                                            const int* __restrict__ active,
                                                            double* __restrict__ part0,
                                                            double* __restrict__ part1) {
  extern __shared__ double th[];
  __shared__ double red[4 * QPB];
  const CsrTile tl = csr_tile(chunks, QPB);
  const unsigned mask = csr_group<QPB>(g, coef, tl.q0, B, active, th);
  if (!mask) return;
  double a0[QPB], a1[QPB];
#pragma unroll
  for (int k = 0; k < QPB; ++k) a0[k] = a1[k] = 0.0;
  auto v = [&](int k, int c) { return z[(size_t)min(tl.q0 + k, B - 1) * y_ld + c]; };
  for (int t = 0; t < kCsrRows; ++t) {
    const int row = tl.chunk * kCsrThreads * kCsrRows + t * kCsrThreads + (int)threadIdx.x;
    if (row >= g.N) continue;
    TY d[QPB], off[QPB];
    csr_row<QPB, TY>(g, row, th, v, d, off);
#pragma unroll
    for (int k = 0; k < QPB; ++k) {
      if (!((mask >> k) & 1u)) continue;
      const TY zi = z[(size_t)(tl.q0 + k) * y_ld + row];
      const double fp = rhs[(size_t)(tl.q0 + k) * rhs_ld + row];
      const TY Az = d[k] * zi + off[k];
      const TY nv = zi + (TY)omega * (((TY)fp - Az) / d[k]);
      y[(size_t)(tl.q0 + k) * y_ld + row] = nv;
      a0[k] += (double)nv * fp;
      if (rhs2) a1[k] += (double)nv * rhs2[(size_t)(tl.q0 + k) * rhs2_ld + row];
    }
  }
  if (part0) csr_partials<QPB>(a0, mask, tl.q0, tl.chunk, chunks, part0, red);
  if (part1) {
    __syncthreads();
    csr_partials<QPB>(a1, mask, tl.q0, tl.chunk, chunks, part1, red);
  }
}

// ---- theta into the per-query tables; storage <-> natural order ---------------------------
__global__ void k_csr_theta(int Q, int ct, const double* __restrict__ theta,
                            const int* __restrict__ qidx, double* __restrict__ coef) {
  const int b = blockIdx.x;
  const int src = qidx ? qidx[b] : b;
  for (int e = threadIdx.x; e < ct; e += blockDim.x)
    coef[(size_t)b * ct + e] = e < Q ? theta[(size_t)src * Q + e] : 0.0;
}

__global__ void k_perm_gather(int N, const int* __restrict__ perm, const double* __restrict__ src,
                              int64_t src_ld, double* __restrict__ dst, int64_t dst_ld) {
  const int b = blockIdx.y;
  for (int pos = blockIdx.x * blockDim.x + threadIdx.x; pos < N; pos += gridDim.x * blockDim.x)
    dst[(size_t)b * dst_ld + pos] = src[(size_t)b * src_ld + perm[pos]];
}
__global__ void k_perm_scatter(int N, const int* __restrict__ perm, const double* __restrict__ src,
                               int64_t src_ld, double* __restrict__ dst, int64_t dst_ld) {
  const int b = blockIdx.y;
  for (int pos = blockIdx.x * blockDim.x + threadIdx.x; pos < N; pos += gridDim.x * blockDim.x)
    dst[(size_t)b * dst_ld + perm[pos]] = src[(size_t)b * src_ld + pos];
}

// ---- launchers (called by the stencil launchers when g.csr is set) -------------------------
static int csr_qpb(int B) { return B >= 4 ? 4 : (B >= 2 ? 2 : 1); }

template <typename F>
static void csr_dispatch(int qpb, F&& f) {
  switch (qpb) {
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 2: f(std::integral_constant<int, 2>{}); break;
    default: f(std::integral_constant<int, 1>{}); break;
  }
}

static dim3 csr_grid(int chunks, int B, int qpb) {
  return dim3((unsigned)((long)chunks * ((B + qpb - 1) / qpb)));
}

void csr_coef_tables(const StencilGeom& g, int B, const double* theta, const int* qidx,
                     double* coef, hipStream_t s) {
  hipLaunchKernelGGL(k_csr_theta, dim3(B), dim3(64), 0, s, g.Q, g.ct_size, theta, qidx, coef);
}

void csr_apply(const StencilGeom& g, int64_t ld, int B, const double* coef, const double* u,
               double* y, int mode, const double* rhs, int64_t rhs_ld, const double* rhs_scale,
               const int* flag, double* part, hipStream_t s, double* part2) {
  const int chunks = csr_chunks(g.N);
  csr_dispatch(csr_qpb(B), [&](auto Q) {
    hipLaunchKernelGGL((k_csr_apply<Q.value>), csr_grid(chunks, B, Q.value), dim3(kCsrThreads),
                       Q.value * g.ct_size * 8, s, g, ld, B, chunks, coef, u, y, mode, rhs,
                       rhs_ld, rhs_scale, flag, part, part2);
  });
}

template <typename TY>
int csr_pass_a(const StencilGeom& g, int64_t ld, int B, const double* coef, const TY* y,
               int64_t y_ld, const double* p_old, double* p_new, const double* beta,
               const int* active, double* part, hipStream_t s) {
  const int chunks = csr_chunks(g.N);
  csr_dispatch(csr_qpb(B), [&](auto Q) {
    hipLaunchKernelGGL((k_csr_pass_a<Q.value, TY>), csr_grid(chunks, B, Q.value),
                       dim3(kCsrThreads), Q.value * g.ct_size * 8, s, g, ld, B, chunks, coef, y,
                       y_ld, p_old, p_new, beta, active, part);
  });
  return chunks;
}
template int csr_pass_a<double>(const StencilGeom&, int64_t, int, const double*, const double*,
                                int64_t, const double*, double*, const double*, const int*,
                                double*, hipStream_t);
template int csr_pass_a<float>(const StencilGeom&, int64_t, int, const double*, const float*,
                               int64_t, const double*, double*, const double*, const int*,
                               double*, hipStream_t);

int csr_pass_b(const StencilGeom& g, int64_t ld, int B, const double* coef, const double* p,
               double* x, const double* r_in, double* r_out, const double* alpha,
               const int* active, double* part, hipStream_t s) {
  const int chunks = csr_chunks(g.N);
  csr_dispatch(csr_qpb(B), [&](auto Q) {
    hipLaunchKernelGGL((k_csr_pass_b<Q.value>), csr_grid(chunks, B, Q.value), dim3(kCsrThreads),
                       Q.value * g.ct_size * 8, s, g, ld, B, chunks, coef, p, x, r_in, r_out,
                       alpha, active, part);
  });
  return chunks;
}

template <typename TY>
void csr_gs_color(const StencilGeom& g, int color, int B, const double* coef, TY* y,
                  int64_t y_ld, const double* rhs, int64_t rhs_ld, const double* rhs_scale,
                  const double* rhs2, int64_t rhs2_ld, const int* active, double* part0,
                  double* part1, hipStream_t s) {
  const int chunks = csr_chunks(g.coff[color + 1] - g.coff[color]);
  if (chunks == 0) return;
  csr_dispatch(csr_qpb(B), [&](auto Q) {
    hipLaunchKernelGGL((k_csr_gs<Q.value, TY>), csr_grid(chunks, B, Q.value), dim3(kCsrThreads),
                       Q.value * g.ct_size * 8, s, g, color, B, chunks, coef, y, y_ld, rhs,
                       rhs_ld, rhs_scale, rhs2, rhs2_ld, active, part0, part1);
  });
}
template void csr_gs_color<double>(const StencilGeom&, int, int, const double*, double*, int64_t,
                                   const double*, int64_t, const double*, const double*, int64_t,
                                   const int*, double*, double*, hipStream_t);
template void csr_gs_color<float>(const StencilGeom&, int, int, const double*, float*, int64_t,
                                  const double*, int64_t, const double*, const double*, int64_t,
                                  const int*, double*, double*, hipStream_t);

template <typename TY>
void csr_jacobi(const StencilGeom& g, int B, const double* coef, const TY* z, TY* y,
                int64_t y_ld, double omega, const double* rhs, int64_t rhs_ld,
                const double* rhs2, int64_t rhs2_ld, const int* active, double* part0,
                double* part1, hipStream_t s) {
  const int chunks = csr_chunks(g.N);
  csr_dispatch(csr_qpb(B), [&](auto Q) {
    hipLaunchKernelGGL((k_csr_jacobi<Q.value, TY>), csr_grid(chunks, B, Q.value),
                       dim3(kCsrThreads), Q.value * g.ct_size * 8, s, g, B, chunks, coef, z, y,
                       y_ld, omega, rhs, rhs_ld, rhs2, rhs2_ld, active, part0, part1);
  });
}
template void csr_jacobi<double>(const StencilGeom&, int, const double*, const double*, double*,
                                 int64_t, double, const double*, int64_t, const double*, int64_t,
                                 const int*, double*, double*, hipStream_t);
template void csr_jacobi<float>(const StencilGeom&, int, const double*, const float*, float*,
                                int64_t, double, const double*, int64_t, const double*, int64_t,
                                const int*, double*, double*, hipStream_t);

static dim3 perm_grid(int N, int B) {
  int bx = (N + 255) / 256;
  if (bx > 4096) bx = 4096;
  return dim3(bx, B);
}
void csr_to_storage(int N, const int* perm, int B, const double* nat, int64_t nat_ld,
                    double* sto, int64_t sto_ld, hipStream_t s) {
  hipLaunchKernelGGL(k_perm_gather, perm_grid(N, B), dim3(256), 0, s, N, perm, nat, nat_ld, sto,
                     sto_ld);
}
void csr_from_storage(int N, const int* perm, int B, const double* sto, int64_t sto_ld,
                      double* nat, int64_t nat_ld, hipStream_t s) {
  hipLaunchKernelGGL(k_perm_scatter, perm_grid(N, B), dim3(256), 0, s, N, perm, sto, sto_ld, nat,
                     nat_ld);
}

}  // namespace rb
