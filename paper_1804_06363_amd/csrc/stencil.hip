// Matrix-free affine block-diffusion operator and the stencil passes of RBCG / RBI.
//
// Operator (eq. 12, Sec. 2.3): A(mu) = sum_q Theta_q(mu) A_q with A_q the finite-
// difference operator of -div(kappa grad u) for kappa = indicator of block q.  For a
// node p, (A u)_p = sum_faces c_f (u_p - u_nb) with c_f = h_a^-2 * (mean of kappa over
// the face's dual cell) and u_nb = 0 outside the grid.  c_f only depends on the block
// of the face along its normal and on the "states" of the node along the two
// tangential axes (inside block t: state 2t; on the interface of blocks t, t+1:
// state 2t+1), so each query gets a small table of face coefficients and every
// node looks up its six faces there.
//
// Vectors are in red-black storage order (see StencilGeom): the red nodes first,
// then the black ones; a node's neighbours all have the other colour and sit at
// constant offsets in the other half, so every pass below reads and writes
// contiguous ranges.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "kernels.h"

namespace rb {

using rbk::fdiv;

// Fraction of a tangential node state s (see above) in block qt.
__device__ __forceinline__ double state_frac(int s, int qt) {
  if ((s & 1) == 0) return (s >> 1) == qt ? 1.0 : 0.0;
  return ((s >> 1) == qt || (s >> 1) + 1 == qt) ? 0.5 : 0.0;
}

// One block per query: coef[b][...] = h_a^-2 * sum_q theta_q * [q_a == bn] *
// frac(s1, q_t1) * frac(s2, q_t2) for every axis a, normal block bn, states s1, s2.
__global__ void k_coef_tables(StencilGeom g, const double* __restrict__ theta,
                              const int* __restrict__ qidx, double* __restrict__ coef,
                              double h2x, double h2y, double h2z) {
  const int b = blockIdx.x;
  const int src = qidx ? qidx[b] : b;
  const double* th = theta + (size_t)src * g.Q;
  double* out = coef + (size_t)b * g.ct_size;
  const int nb[3] = {g.bx, g.by, g.bz};
  const double h2[3] = {h2x, h2y, h2z};
  for (int a = 0; a < g.dim; ++a) {
    const int t1 = a == 0 ? 1 : 0;
    const int t2 = a == 2 ? 1 : 2;
    const int s1n = g.ct_s1[a], s2n = g.ct_s2[a];
    const int cnt = nb[a] * s1n * s2n;
    for (int e = threadIdx.x; e < cnt; e += blockDim.x) {
      const int s2 = e % s2n;
      const int s1 = (e / s2n) % s1n;
      const int bn = e / (s1n * s2n);
      double acc = 0.0;
      for (int q = 0; q < g.Q; ++q) {
        int qc[3];
        qc[0] = q % g.bx;
        qc[1] = (q / g.bx) % g.by;
        qc[2] = q / (g.bx * g.by);
        if (qc[a] != bn) continue;
        const double w = state_frac(s1, qc[t1]) * state_frac(s2, qc[t2]);
        acc += th[q] * w;
      }
      out[g.ct_off[a] + e] = acc * h2[a];
    }
  }
  // padding
  for (int e = g.ct_off[g.dim - 1] + nb[g.dim - 1] * g.ct_s1[g.dim - 1] * g.ct_s2[g.dim - 1] +
               threadIdx.x;
       e < g.ct_size; e += blockDim.x)
    out[e] = 0.0;
}

void launch_coef_tables(const StencilGeom& g, int B, const double* theta, const int* qidx,
                        double* coef, hipStream_t s) {
  const double hx = 1.0 / (g.nx + 1), hy = 1.0 / (g.ny + 1), hz = 1.0 / (g.nz + 1);
  hipLaunchKernelGGL(k_coef_tables, dim3(B), dim3(64), 0, s, g, theta, qidx, coef,
                     1.0 / (hx * hx), 1.0 / (hy * hy), 1.0 / (hz * hz));
}

// ---- per-node stencil geometry ---------------------------------------------------
template <int DIM>
struct Node {
  int L;            // lexicographic index
  int nb[2 * DIM];  // storage positions of the neighbours (-1: boundary)
  int ci[2 * DIM];  // coefficient-table index of each face
};

template <int DIM>
__device__ __forceinline__ void node_at(const StencilGeom& g, int pos, Node<DIM>& n) {
  const int c = pos >= g.NR;
  const int L = c ? 2 * (pos - g.NR) + 1 : 2 * pos;
  n.L = L;
  const int other = c ? 0 : g.NR;
  int i, j = 0, k = 0;
  if (DIM == 1) {
    i = L;
  } else if (DIM == 2) {
    j = (int)fdiv((uint32_t)L, g.div_nx);
    i = L - j * g.nx;
  } else {
    k = (int)fdiv((uint32_t)L, g.div_nxy);
    const int rem = L - k * g.nxy;
    j = (int)fdiv((uint32_t)rem, g.div_nx);
    i = rem - j * g.nx;
  }
  const uint32_t tx = g.tab[0][i];
  const uint32_t ty = DIM >= 2 ? g.tab[1][j] : 0u;
  const uint32_t tz = DIM >= 3 ? g.tab[2][k] : 0u;
  const int sx = tx & 0xff, sy = ty & 0xff, sz = tz & 0xff;
  // x faces: tangential (y, z)
  n.ci[0] = g.ct_off[0] + ((int)((tx >> 8) & 0xff) * g.ct_s1[0] + sy) * g.ct_s2[0] + sz;
  n.ci[1] = g.ct_off[0] + ((int)((tx >> 16) & 0xff) * g.ct_s1[0] + sy) * g.ct_s2[0] + sz;
  n.nb[0] = i > 0 ? other + ((L - 1) >> 1) : -1;
  n.nb[1] = i < g.nx - 1 ? other + ((L + 1) >> 1) : -1;
  if (DIM >= 2) {  // y faces: tangential (x, z)
    n.ci[2] = g.ct_off[1] + ((int)((ty >> 8) & 0xff) * g.ct_s1[1] + sx) * g.ct_s2[1] + sz;
    n.ci[3] = g.ct_off[1] + ((int)((ty >> 16) & 0xff) * g.ct_s1[1] + sx) * g.ct_s2[1] + sz;
    n.nb[2] = j > 0 ? other + ((L - g.nx) >> 1) : -1;
    n.nb[3] = j < g.ny - 1 ? other + ((L + g.nx) >> 1) : -1;
  }
  if (DIM >= 3) {  // z faces: tangential (x, y)
    n.ci[4] = g.ct_off[2] + ((int)((tz >> 8) & 0xff) * g.ct_s1[2] + sx) * g.ct_s2[2] + sy;
    n.ci[5] = g.ct_off[2] + ((int)((tz >> 16) & 0xff) * g.ct_s1[2] + sx) * g.ct_s2[2] + sy;
    n.nb[4] = k > 0 ? other + ((L - g.nxy) >> 1) : -1;
    n.nb[5] = k < g.nz - 1 ? other + ((L + g.nxy) >> 1) : -1;
  }
}

// (A v)_p given a functor V(pos) returning the vector value at a storage position.
template <int DIM, typename T, typename V>
__device__ __forceinline__ T apply_at(const Node<DIM>& n, const T* __restrict__ cf, T vp,
                                      V val, T& diag) {
  T d = T(0), off = T(0);
#pragma unroll
  for (int f = 0; f < 2 * DIM; ++f) {
    const T c = cf[n.ci[f]];
    d += c;
    if (n.nb[f] >= 0) off += c * val(n.nb[f]);
  }
  diag = d;
  return d * vp - off;
}

// Loads the query's coefficient table into LDS (as T).
template <typename T>
__device__ __forceinline__ void load_coef(const StencilGeom& g, const double* coef, int b,
                                          T* sh) {
  const double* src = coef + (size_t)b * g.ct_size;
  for (int e = threadIdx.x; e < g.ct_size; e += blockDim.x) sh[e] = (T)src[e];
  __syncthreads();
}

constexpr int kThreads = 256;
constexpr int kMaxCoef = 1024;  // doubles per query table (host checks)

// ---- y = A(theta) u, plus optional ||rhs - A u||^2 ------------------------------
// Grid: (chunks, B).  mode 0: y = A u.  mode 1: y = rhs - A u for queries with
// flag[b] != 0 (others skipped), partial sums of y^2 in part[b][chunk].
template <int DIM>
__global__ __launch_bounds__(kThreads) void k_apply(StencilGeom g, int64_t ld, const double* coef,
                                                    const double* __restrict__ u,
                                                    double* __restrict__ y, int mode,
                                                    const double* __restrict__ rhs,
                                                    int64_t rhs_ld, const double* __restrict__ rhs_scale,
                                                    const int* __restrict__ flag,
                                                    double* __restrict__ part, int per_thread) {
  __shared__ double cf[kMaxCoef];
  __shared__ double red[4];
  const int b = blockIdx.y;
  if (mode == 1 && flag[b] == 0) return;
  load_coef(g, coef, b, cf);
  const double* ub = u + (size_t)b * ld;
  double* yb = y + (size_t)b * ld;
  const double* fb = mode == 1 ? rhs + (size_t)b * rhs_ld : nullptr;
  const double fs = mode == 1 ? rhs_scale[b] : 0.0;
  double acc = 0.0;
  const int base = blockIdx.x * kThreads * per_thread;
  for (int t = 0; t < per_thread; ++t) {
    const int pos = base + t * kThreads + threadIdx.x;
    if (pos >= g.N) break;
    Node<DIM> n;
    node_at<DIM>(g, pos, n);
    double d;
    const double Au = apply_at<DIM, double>(n, cf, ub[pos], [&](int q) { return ub[q]; }, d);
    if (mode == 0) {
      yb[pos] = Au;
    } else {
      const double r = fs * fb[pos] - Au;
      yb[pos] = r;
      acc += r * r;
    }
  }
  if (mode == 1) {
    const double s = rbk::block_sum_256(acc, red);
    if (threadIdx.x == 0) part[(size_t)b * gridDim.x + blockIdx.x] = s;
  }
}

// ---- pass A: p_new = y + beta p_old; q = A p_new; partial p_new^T q -------------
template <int DIM, typename TY>
__global__ __launch_bounds__(kThreads) void k_pass_a(StencilGeom g, int64_t ld, const double* coef,
                                                     const TY* __restrict__ y, int64_t y_ld,
                                                     const double* __restrict__ p_old,
                                                     double* __restrict__ p_new,
                                                     const double* __restrict__ beta,
                                                     const int* __restrict__ active,
                                                     double* __restrict__ part, int per_thread) {
  __shared__ double cf[kMaxCoef];
  __shared__ double red[4];
  const int b = blockIdx.y;
  if (!active[b]) return;
  load_coef(g, coef, b, cf);
  const double be = beta[b];
  const TY* yb = y + (size_t)b * y_ld;
  const double* po = p_old + (size_t)b * ld;
  double* pn = p_new + (size_t)b * ld;
  double acc = 0.0;
  const int base = blockIdx.x * kThreads * per_thread;
  for (int t = 0; t < per_thread; ++t) {
    const int pos = base + t * kThreads + threadIdx.x;
    if (pos >= g.N) break;
    Node<DIM> n;
    node_at<DIM>(g, pos, n);
    const double pp = (double)yb[pos] + be * po[pos];
    double d;
    const double q = apply_at<DIM, double>(
        n, cf, pp, [&](int s) { return (double)yb[s] + be * po[s]; }, d);
    pn[pos] = pp;
    acc += pp * q;
  }
  const double s = rbk::block_sum_256(acc, red);
  if (threadIdx.x == 0) part[(size_t)b * gridDim.x + blockIdx.x] = s;
}

// ---- pass B: x += alpha p; r_out = r_in - alpha A p; partial ||r_out||^2 ----------
template <int DIM>
__global__ __launch_bounds__(kThreads) void k_pass_b(StencilGeom g, int64_t ld, const double* coef,
                                                     const double* __restrict__ p,
                                                     double* __restrict__ x,
                                                     const double* r_in, double* r_out,
                                                     const double* __restrict__ alpha,
                                                     const int* __restrict__ active,
                                                     double* __restrict__ part, int per_thread) {
  __shared__ double cf[kMaxCoef];
  __shared__ double red[4];
  const int b = blockIdx.y;
  if (!active[b]) return;
  load_coef(g, coef, b, cf);
  const double al = alpha[b];
  const double* pb = p + (size_t)b * ld;
  double* xb = x + (size_t)b * ld;
  const double* ri = r_in + (size_t)b * ld;
  double* ro = r_out + (size_t)b * ld;
  double acc = 0.0;
  const int base = blockIdx.x * kThreads * per_thread;
  for (int t = 0; t < per_thread; ++t) {
    const int pos = base + t * kThreads + threadIdx.x;
    if (pos >= g.N) break;
    Node<DIM> n;
    node_at<DIM>(g, pos, n);
    const double pp = pb[pos];
    double d;
    const double q = apply_at<DIM, double>(n, cf, pp, [&](int s) { return pb[s]; }, d);
    xb[pos] += al * pp;
    const double r = ri[pos] - al * q;
    ro[pos] = r;
    acc += r * r;
  }
  const double s = rbk::block_sum_256(acc, red);
  if (threadIdx.x == 0) part[(size_t)b * gridDim.x + blockIdx.x] = s;
}

// ---- one colour half-sweep of Gauss-Seidel on A y = rhs ---------------------------
// For every node of colour `color`: y_p = (rhs_p - sum_nb A_p,nb y_nb) / A_pp with
// A_p,nb = -c_f (the neighbours all have the other colour).  rhs_b = rhs_scale[b] * rhs[b*rhs_ld + p].
// Partial sums over the updated nodes: y_p rhs_p (dot0) and y_p rhs2_p (dot1).
template <int DIM, typename TY>
__global__ __launch_bounds__(kThreads) void k_gs_color(StencilGeom g, int color, const double* coef,
                                                       TY* __restrict__ y, int64_t y_ld,
                                                       const double* __restrict__ rhs, int64_t rhs_ld,
                                                       const double* __restrict__ rhs_scale,
                                                       const double* __restrict__ rhs2,
                                                       int64_t rhs2_ld,
                                                       const int* __restrict__ active,
                                                       double* __restrict__ part0,
                                                       double* __restrict__ part1,
                                                       int per_thread) {
  using TC = TY;  // coefficient arithmetic in the smoother's precision
  __shared__ TC cf[kMaxCoef];
  __shared__ double red[4];
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  load_coef(g, coef, b, cf);
  TY* yb = y + (size_t)b * y_ld;
  const double* fb = rhs + (size_t)b * rhs_ld;
  const double fs = rhs_scale ? rhs_scale[b] : 1.0;
  const double* f2 = rhs2 ? rhs2 + (size_t)b * rhs2_ld : nullptr;
  const int lo = color ? g.NR : 0;
  const int hi = color ? g.N : g.NR;
  double a0 = 0.0, a1 = 0.0;
  const int base = lo + blockIdx.x * kThreads * per_thread;
  for (int t = 0; t < per_thread; ++t) {
    const int pos = base + t * kThreads + threadIdx.x;
    if (pos >= hi) break;
    Node<DIM> n;
    node_at<DIM>(g, pos, n);
    TC d = TC(0), off = TC(0);
#pragma unroll
    for (int f = 0; f < 2 * DIM; ++f) {
      const TC c = cf[n.ci[f]];
      d += c;
      if (n.nb[f] >= 0) off += c * yb[n.nb[f]];
    }
    // the off-diagonal entries of A are -c: y_p = (rhs_p + sum_nb c y_nb) / d_p
    const double fp = fs * fb[pos];
    const TY v = (TY)(((TC)fp + off) / d);
    yb[pos] = v;
    a0 += (double)v * fp;
    if (f2) a1 += (double)v * f2[pos];
  }
  if (part0) {
    const double s0 = rbk::block_sum_256(a0, red);
    if (threadIdx.x == 0) part0[(size_t)b * gridDim.x + blockIdx.x] = s0;
  }
  if (part1) {
    const double s1 = rbk::block_sum_256(a1, red);
    if (threadIdx.x == 0) part1[(size_t)b * gridDim.x + blockIdx.x] = s1;
  }
}

// ---- damped Jacobi: y = z + omega D^-1 (rhs - A z), partial y^T rhs (and y^T rhs2)
template <int DIM, typename TY>
__global__ __launch_bounds__(kThreads) void k_jacobi(StencilGeom g, const double* coef,
                                                     const TY* __restrict__ z, TY* __restrict__ y,
                                                     int64_t y_ld, double omega,
                                                     const double* __restrict__ rhs, int64_t rhs_ld,
                                                     const double* __restrict__ rhs2, int64_t rhs2_ld,
                                                     const int* __restrict__ active,
                                                     double* __restrict__ part0,
                                                     double* __restrict__ part1, int per_thread) {
  __shared__ TY cf[kMaxCoef];
  __shared__ double red[4];
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  load_coef(g, coef, b, cf);
  const TY* zb = z + (size_t)b * y_ld;
  TY* yb = y + (size_t)b * y_ld;
  const double* fb = rhs + (size_t)b * rhs_ld;
  const double* f2 = rhs2 ? rhs2 + (size_t)b * rhs2_ld : nullptr;
  double a0 = 0.0, a1 = 0.0;
  const int base = blockIdx.x * kThreads * per_thread;
  for (int t = 0; t < per_thread; ++t) {
    const int pos = base + t * kThreads + threadIdx.x;
    if (pos >= g.N) break;
    Node<DIM> n;
    node_at<DIM>(g, pos, n);
    TY d;
    const TY Az = apply_at<DIM, TY>(n, cf, zb[pos], [&](int s) { return zb[s]; }, d);
    const double fp = fb[pos];
    const TY v = zb[pos] + (TY)omega * (((TY)fp - Az) / d);
    yb[pos] = v;
    a0 += (double)v * fp;
    if (f2) a1 += (double)v * f2[pos];
  }
  if (part0) {
    const double s0 = rbk::block_sum_256(a0, red);
    if (threadIdx.x == 0) part0[(size_t)b * gridDim.x + blockIdx.x] = s0;
  }
  if (part1) {
    const double s1 = rbk::block_sum_256(a1, red);
    if (threadIdx.x == 0) part1[(size_t)b * gridDim.x + blockIdx.x] = s1;
  }
}

// ---- natural <-> red-black storage order -------------------------------------------
__global__ void k_to_storage(int N, int NR, const double* __restrict__ nat, int64_t nat_ld,
                             double* __restrict__ sto, int64_t sto_ld) {
  const int b = blockIdx.y;
  for (int pos = blockIdx.x * blockDim.x + threadIdx.x; pos < N; pos += gridDim.x * blockDim.x) {
    const int L = pos < NR ? 2 * pos : 2 * (pos - NR) + 1;
    sto[(size_t)b * sto_ld + pos] = nat[(size_t)b * nat_ld + L];
  }
}
__global__ void k_from_storage(int N, int NR, const double* __restrict__ sto, int64_t sto_ld,
                               double* __restrict__ nat, int64_t nat_ld) {
  const int b = blockIdx.y;
  for (int pos = blockIdx.x * blockDim.x + threadIdx.x; pos < N; pos += gridDim.x * blockDim.x) {
    const int L = pos < NR ? 2 * pos : 2 * (pos - NR) + 1;
    nat[(size_t)b * nat_ld + L] = sto[(size_t)b * sto_ld + pos];
  }
}

static dim3 conv_grid(int N, int B) {
  int bx = (N + 255) / 256;
  if (bx > 4096) bx = 4096;
  return dim3(bx, B);
}

void launch_to_storage(const rb_problem& p, int B, const double* nat, int64_t nat_ld,
                       double* sto, int64_t sto_ld, hipStream_t s) {
  hipLaunchKernelGGL(k_to_storage, conv_grid(p.g.N, B), dim3(256), 0, s, p.g.N, p.g.NR, nat,
                     nat_ld, sto, sto_ld);
}
void launch_from_storage(const rb_problem& p, int B, const double* sto, int64_t sto_ld,
                         double* nat, int64_t nat_ld, hipStream_t s) {
  hipLaunchKernelGGL(k_from_storage, conv_grid(p.g.N, B), dim3(256), 0, s, p.g.N, p.g.NR, sto,
                     sto_ld, nat, nat_ld);
}

// ---- launchers -----------------------------------------------------------------------
int stencil_chunks(int count, int per_thread) {
  const int per_block = kThreads * per_thread;
  return (count + per_block - 1) / per_block;
}

#define RB_DIM_DISPATCH(dim, F) \
  switch (dim) {                \
    case 1: F(1); break;        \
    case 2: F(2); break;        \
    default: F(3); break;       \
  }

void launch_apply(const StencilGeom& g, int64_t ld, int B, const double* coef, const double* u,
                  double* y, int mode, const double* rhs, int64_t rhs_ld, const double* rhs_scale,
                  const int* flag, double* part, int per_thread, hipStream_t s) {
  const dim3 grid(stencil_chunks(g.N, per_thread), B);
#define F(D)                                                                                 \
  hipLaunchKernelGGL(k_apply<D>, grid, dim3(kThreads), 0, s, g, ld, coef, u, y, mode, rhs, \
                     rhs_ld, rhs_scale, flag, part, per_thread)
  RB_DIM_DISPATCH(g.dim, F)
#undef F
}

template <typename TY>
void launch_pass_a(const StencilGeom& g, int64_t ld, int B, const double* coef, const TY* y,
                   int64_t y_ld, const double* p_old, double* p_new, const double* beta,
                   const int* active, double* part, int per_thread, hipStream_t s) {
  const dim3 grid(stencil_chunks(g.N, per_thread), B);
#define F(D)                                                                               \
  hipLaunchKernelGGL((k_pass_a<D, TY>), grid, dim3(kThreads), 0, s, g, ld, coef, y, y_ld, \
                     p_old, p_new, beta, active, part, per_thread)
  RB_DIM_DISPATCH(g.dim, F)
#undef F
}
template void launch_pass_a<double>(const StencilGeom&, int64_t, int, const double*,
                                    const double*, int64_t, const double*, double*,
                                    const double*, const int*, double*, int, hipStream_t);
template void launch_pass_a<float>(const StencilGeom&, int64_t, int, const double*, const float*,
                                   int64_t, const double*, double*, const double*, const int*,
                                   double*, int, hipStream_t);

void launch_pass_b(const StencilGeom& g, int64_t ld, int B, const double* coef, const double* p,
                   double* x, const double* r_in, double* r_out, const double* alpha,
                   const int* active, double* part, int per_thread, hipStream_t s) {
  const dim3 grid(stencil_chunks(g.N, per_thread), B);
#define F(D)                                                                                \
  hipLaunchKernelGGL(k_pass_b<D>, grid, dim3(kThreads), 0, s, g, ld, coef, p, x, r_in, r_out, \
                     alpha, active, part, per_thread)
  RB_DIM_DISPATCH(g.dim, F)
#undef F
}

template <typename TY>
void launch_gs_color(const StencilGeom& g, int color, int B, const double* coef, TY* y,
                     int64_t y_ld, const double* rhs, int64_t rhs_ld, const double* rhs_scale,
                     const double* rhs2, int64_t rhs2_ld, const int* active, double* part0,
                     double* part1, int per_thread, hipStream_t s) {
  const int count = color ? g.N - g.NR : g.NR;
  const dim3 grid(stencil_chunks(count, per_thread), B);
#define F(D)                                                                                  \
  hipLaunchKernelGGL((k_gs_color<D, TY>), grid, dim3(kThreads), 0, s, g, color, coef, y, y_ld, \
                     rhs, rhs_ld, rhs_scale, rhs2, rhs2_ld, active, part0, part1, per_thread)
  RB_DIM_DISPATCH(g.dim, F)
#undef F
}
template void launch_gs_color<double>(const StencilGeom&, int, int, const double*, double*,
                                      int64_t, const double*, int64_t, const double*,
                                      const double*, int64_t, const int*, double*, double*, int,
                                      hipStream_t);
template void launch_gs_color<float>(const StencilGeom&, int, int, const double*, float*, int64_t,
                                     const double*, int64_t, const double*, const double*,
                                     int64_t, const int*, double*, double*, int, hipStream_t);

template <typename TY>
void launch_jacobi(const StencilGeom& g, int B, const double* coef, const TY* z, TY* y,
                   int64_t y_ld, double omega, const double* rhs, int64_t rhs_ld,
                   const double* rhs2, int64_t rhs2_ld, const int* active, double* part0,
                   double* part1, int per_thread, hipStream_t s) {
  const dim3 grid(stencil_chunks(g.N, per_thread), B);
#define F(D)                                                                                   \
  hipLaunchKernelGGL((k_jacobi<D, TY>), grid, dim3(kThreads), 0, s, g, coef, z, y, y_ld, omega, \
                     rhs, rhs_ld, rhs2, rhs2_ld, active, part0, part1, per_thread)
  RB_DIM_DISPATCH(g.dim, F)
#undef F
}
template void launch_jacobi<double>(const StencilGeom&, int, const double*, const double*,
                                    double*, int64_t, double, const double*, int64_t,
                                    const double*, int64_t, const int*, double*, double*, int,
                                    hipStream_t);
template void launch_jacobi<float>(const StencilGeom&, int, const double*, const float*, float*,
                                   int64_t, double, const double*, int64_t, const double*,
                                   int64_t, const int*, double*, double*, int, hipStream_t);

}  // namespace rb
