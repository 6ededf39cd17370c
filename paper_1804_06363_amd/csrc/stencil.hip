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

#include <algorithm>
#include <type_traits>

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
  if (g.csr) return csr_coef_tables(g, B, theta, qidx, coef, s);
  const double hx = 1.0 / (g.nx + 1), hy = 1.0 / (g.ny + 1), hz = 1.0 / (g.nz + 1);
  hipLaunchKernelGGL(k_coef_tables, dim3(B), dim3(64), 0, s, g, theta, qidx, coef,
                     1.0 / (hx * hx), 1.0 / (hy * hy), 1.0 / (hz * hz));
}

// ---- per-node stencil geometry ---------------------------------------------------
// nb[f] is the storage position of the neighbour across face f; at the boundary it is
// the node itself (a valid address) and bit f of `inner` is clear, so the loaded value
// is replaced by zero instead of the load being branched around: all the loads of a
// node can be in flight together.
template <int DIM>
struct Node {
  int nb[2 * DIM];  // storage positions of the neighbours (self at the boundary)
  int ci[2 * DIM];  // coefficient-table index of each face
  unsigned inner;   // bit f: face f has an interior neighbour
};

template <int DIM>
__device__ __forceinline__ void node_at(const StencilGeom& g, int pos, Node<DIM>& n) {
  const int c = pos >= g.NR;
  const int L = c ? 2 * (pos - g.NR) + 1 : 2 * pos;
  const int other = c ? 0 : g.NR;
  int i, j = 0, k = 0;
  if constexpr (DIM == 1) {
    i = L;
  } else if constexpr (DIM == 2) {
    j = (int)fdiv((uint32_t)L, g.div_nx);
    i = L - j * g.nx;
  } else {
    k = (int)fdiv((uint32_t)L, g.div_nxy);
    const int rem = L - k * g.nxy;
    j = (int)fdiv((uint32_t)rem, g.div_nx);
    i = rem - j * g.nx;
  }
  const uint32_t tx = g.tab[0][i];
  uint32_t ty = 0u, tz = 0u;
  if constexpr (DIM >= 2) ty = g.tab[1][j];
  if constexpr (DIM >= 3) tz = g.tab[2][k];
  const int sx = tx & 0xff, sy = ty & 0xff, sz = tz & 0xff;
  unsigned inner = 0;
  // x faces: tangential (y, z)
  n.ci[0] = g.ct_off[0] + ((int)((tx >> 8) & 0xff) * g.ct_s1[0] + sy) * g.ct_s2[0] + sz;
  n.ci[1] = g.ct_off[0] + ((int)((tx >> 16) & 0xff) * g.ct_s1[0] + sy) * g.ct_s2[0] + sz;
  const bool xl = i > 0, xh = i < g.nx - 1;
  n.nb[0] = xl ? other + ((L - 1) >> 1) : pos;
  n.nb[1] = xh ? other + ((L + 1) >> 1) : pos;
  inner |= (xl ? 1u : 0u) | (xh ? 2u : 0u);
  if constexpr (DIM >= 2) {  // y faces: tangential (x, z)
    n.ci[2] = g.ct_off[1] + ((int)((ty >> 8) & 0xff) * g.ct_s1[1] + sx) * g.ct_s2[1] + sz;
    n.ci[3] = g.ct_off[1] + ((int)((ty >> 16) & 0xff) * g.ct_s1[1] + sx) * g.ct_s2[1] + sz;
    const bool yl = j > 0, yh = j < g.ny - 1;
    n.nb[2] = yl ? other + ((L - g.nx) >> 1) : pos;
    n.nb[3] = yh ? other + ((L + g.nx) >> 1) : pos;
    inner |= (yl ? 4u : 0u) | (yh ? 8u : 0u);
  }
  if constexpr (DIM >= 3) {  // z faces: tangential (x, y)
    n.ci[4] = g.ct_off[2] + ((int)((tz >> 8) & 0xff) * g.ct_s1[2] + sx) * g.ct_s2[2] + sy;
    n.ci[5] = g.ct_off[2] + ((int)((tz >> 16) & 0xff) * g.ct_s1[2] + sx) * g.ct_s2[2] + sy;
    const bool zl = k > 0, zh = k < g.nz - 1;
    n.nb[4] = zl ? other + ((L - g.nxy) >> 1) : pos;
    n.nb[5] = zh ? other + ((L + g.nxy) >> 1) : pos;
    inner |= (zl ? 16u : 0u) | (zh ? 32u : 0u);
  }
  n.inner = inner;
}

// (A v)_p given a functor V(pos) returning the vector value at a storage position.
template <int DIM, typename T, typename V>
__device__ __forceinline__ T apply_at(const Node<DIM>& n, const T* __restrict__ cf, T vp,
                                      V val, T& diag) {
  T vals[2 * DIM];
#pragma unroll
  for (int f = 0; f < 2 * DIM; ++f) vals[f] = val(n.nb[f]);
  T d = T(0), off = T(0);
#pragma unroll
  for (int f = 0; f < 2 * DIM; ++f) {
    const T c = cf[n.ci[f]];
    d += c;
    // select the value, not the coefficient: the self-load at the boundary may hold
    // anything (0 * NaN would poison the sum)
    off += c * (((n.inner >> f) & 1u) ? vals[f] : T(0));
  }
  diag = d;
  return d * vp - off;
}

// y = num / d in the smoother's precision.  FP32: the hardware reciprocal refined by one
// Newton step on the quotient (q = num r, q += r (num - d q)), within an ulp of the
// rounded quotient in a third of the instructions of the IEEE sequence (d > 0 is a sum of
// face coefficients); FP64: IEEE division.  Every stencil sweep kernel uses it, so they
// agree bit for bit.
template <typename T>
__device__ __forceinline__ T gs_div(T num, T d) {
  if constexpr (sizeof(T) == 4) {
    const float r = __builtin_amdgcn_rcpf(d);
    const float q = num * r;
    return __builtin_fmaf(__builtin_fmaf(-d, q, num), r, q);
  } else {
    return num / d;
  }
}

// the element `byte_off` bytes past a block-uniform base: a scalar base plus a 32-bit
// vector offset per load (rows are far below 4 GiB)
template <typename T>
__device__ __forceinline__ const T& at_byte(const T* base, uint32_t byte_off) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + byte_off);
}
template <typename T>
__device__ __forceinline__ T& at_byte(T* base, uint32_t byte_off) {
  return *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + byte_off);
}

// ---- batched pass kernels -------------------------------------------------------------
// Every pass below runs on a 1D grid of (query group) x (node chunk) blocks.  A block
// owns QPB consecutive queries and kPT*256 consecutive storage positions: each thread
// decodes the geometry of its nodes once and applies it to the QPB queries (their
// loads are independent, which keeps many requests in flight).  Block ids are
// remapped so that each XCD (blocks are dealt round-robin to the 8 XCDs) streams one
// contiguous range of (group, chunk) pairs and finds the row/plane neighbours of its
// nodes in its own L2.  Partial sums go to part[b][chunk] (stride = chunks).
constexpr int kThreads = 256;
#ifndef RB_KPT
#define RB_KPT 4
#endif
#ifndef RB_KPH
#define RB_KPH 2
#endif
#ifndef RB_QPB_MAX
#define RB_QPB_MAX 8
#endif
constexpr int kPT = RB_KPT;  // positions per thread in the one-colour passes
constexpr int kPH = RB_KPH;  // positions per thread and colour in the all-node passes
constexpr int kXCD = 8;

// All-node passes: chunk c holds red positions [c*CH, (c+1)*CH) and the black positions
// NRa + [c*CH, (c+1)*CH) (CH = 256*kPH; NRa = NR rounded down to a multiple of 32, the
// positions below NR left out), so the red and black neighbours of a node are loaded by
// the same block and the plane neighbours by the chunks next to it, and every wave's run
// of black positions starts on a 128-byte line (NR is odd on odd 2D grids).
constexpr int kAlign = 32;  // positions per 128-byte line of FP32 values
__device__ __forceinline__ int paired_pos(const StencilGeom& g, int chunk, int t) {
  const int half = t / kPH, u = t % kPH;
  const int off = chunk * kThreads * kPH + u * kThreads + (int)threadIdx.x;
  if (half == 0) return off < g.NR ? off : -1;
  const int b = (g.NR & ~(kAlign - 1)) + off;
  return (b >= g.NR && b < g.N) ? b : -1;
}

__device__ __forceinline__ int xcd_remap(int b, int total) {
#ifdef RB_NO_XCD_REMAP
  return b;
#endif
  const int q = total / kXCD, r = total % kXCD;
  const int xcd = b % kXCD, slot = b / kXCD;
  return xcd < r ? xcd * (q + 1) + slot : r * (q + 1) + (xcd - r) * q + slot;
}

struct Tile {
  int chunk, q0;
};
__device__ __forceinline__ Tile tile_of(int chunks) {
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  return Tile{blk % chunks, (blk / chunks)};
}

// Loads the coefficient tables of queries q0..q0+QPB-1 into LDS (as T); returns the
// mask of queries that exist and are active.
template <int QPB, typename T>
__device__ __forceinline__ unsigned load_group(const StencilGeom& g, const double* coef, int q0,
                                               int B, const int* active, T* sh) {
  unsigned mask = 0;
#pragma unroll
  for (int k = 0; k < QPB; ++k) {
    const int b = q0 + k;
    if (b < B && (!active || active[b])) mask |= 1u << k;
  }
  if (mask)
    for (int e = threadIdx.x; e < QPB * g.ct_size; e += blockDim.x) {
      const int k = e / g.ct_size;
      sh[e] = (q0 + k < B) ? (T)coef[(size_t)(q0 + k) * g.ct_size + (e - k * g.ct_size)] : T(0);
    }
  __syncthreads();
  return mask;
}

template <int QPB>
__device__ __forceinline__ void store_partials(const double (&acc)[QPB], unsigned mask, int q0,
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

template <int DIM, typename T>
__device__ __forceinline__ T diag_of(const Node<DIM>& n, const T* cf) {
  T d = T(0);
#pragma unroll
  for (int f = 0; f < 2 * DIM; ++f) d += cf[n.ci[f]];
  return d;
}

// ---- y = A(theta) u, or y = rhs - A u with partial ||y||^2 ------------------------------
// mode 0: y = A u for every query.  mode 1: y = rhs_scale[b] * rhs_b - A u for queries
// with flag[b] != 0 (others untouched) and partial sums of y^2; y32 (nullable, mode 1):
// an FP32 copy of y, rows of ld.
// group bitmap of the apply kernel: at most kApplyMaxGroupWords * 32 = 16384 groups per
// block (the launcher adds slots beyond that; batches hold at most 65535 queries)
constexpr int kApplyMaxGroupWords = 512;

template <int DIM, int QPB>
__global__ __launch_bounds__(kThreads) void k_apply(StencilGeom g, int64_t ld, int B, int chunks,
                                                    const double* coef,
                                                    const double* __restrict__ u,
                                                    double* __restrict__ y, int mode,
                                                    const double* __restrict__ rhs,
                                                    int64_t rhs_ld,
                                                    const double* __restrict__ rhs_scale,
                                                    const int* __restrict__ flag,
                                                    double* __restrict__ part,
                                                    double* __restrict__ part2,
                                                    float* __restrict__ y32) {
  extern __shared__ double dyn[];
  __shared__ double red[4 * QPB];
  // A block owns one chunk and the query groups slot, slot + slots, ...: with few slots
  // an all-but-empty launch (mode 1 with few flagged queries) costs few blocks.  Mode 1
  // first marks the groups holding a flagged query (one pass over the flags), then
  // visits only those.
  __shared__ unsigned gbits[kApplyMaxGroupWords];
  const Tile tl = tile_of(chunks);
  const int slots = gridDim.x / chunks;
  const int groups = (B + QPB - 1) / QPB;
  const int mine = (groups - tl.q0 + slots - 1) / slots;  // groups of this block
  if (mode == 1) {
    for (int w = threadIdx.x; w < (mine + 31) / 32; w += blockDim.x) gbits[w] = 0u;
    __syncthreads();
    for (int i = threadIdx.x; i < mine * QPB; i += blockDim.x) {
      const int b = (tl.q0 + (i / QPB) * slots) * QPB + i % QPB;
      if (b < B && flag[b]) atomicOr(&gbits[(i / QPB) >> 5], 1u << ((i / QPB) & 31));
    }
    __syncthreads();
  }
  for (int k_ = 0; k_ < mine; ++k_) {
    if (mode == 1 && !((gbits[k_ >> 5] >> (k_ & 31)) & 1u)) continue;
    const int grp = tl.q0 + k_ * slots;
    const int q0 = grp * QPB;
    const unsigned mask = load_group<QPB>(g, coef, q0, B, mode == 1 ? flag : nullptr, dyn);
    if (!mask) continue;
    double acc[QPB], acc2[QPB];
#pragma unroll
    for (int k = 0; k < QPB; ++k) acc[k] = acc2[k] = 0.0;
#pragma unroll
    for (int t = 0; t < 2 * kPH; ++t) {
      const int pos = paired_pos(g, tl.chunk, t);
      if (pos >= 0) {
        Node<DIM> n;
        node_at<DIM>(g, pos, n);
#pragma unroll
        for (int k = 0; k < QPB; ++k) {
          if (!((mask >> k) & 1u)) continue;
          const double* cf = dyn + k * g.ct_size;
          const double* ub = u + (size_t)(q0 + k) * ld;
          double d;
          const double Au =
              apply_at<DIM, double>(n, cf, ub[pos], [&](int s) { return ub[s]; }, d);
          if (mode == 0) {
            y[(size_t)(q0 + k) * ld + pos] = Au;
          } else {
            const double r = rhs_scale[q0 + k] * rhs[(size_t)(q0 + k) * rhs_ld + pos] - Au;
            y[(size_t)(q0 + k) * ld + pos] = r;
            if (y32) y32[(size_t)(q0 + k) * ld + pos] = (float)r;
            acc[k] += r * r;
            if (part2) {  // (|A| |u|)_pos: the face coefficients are non-negative
              double a = d * fabs(ub[pos]);
#pragma unroll
              for (int f = 0; f < 2 * DIM; ++f)
                a += cf[n.ci[f]] * (((n.inner >> f) & 1u) ? fabs(ub[n.nb[f]]) : 0.0);
              acc2[k] += a * a;
            }
          }
        }
      }
    }
    if (mode == 1) store_partials<QPB>(acc, mask, q0, tl.chunk, chunks, part, red);
    if (mode == 1 && part2) {
      __syncthreads();
      store_partials<QPB>(acc2, mask, q0, tl.chunk, chunks, part2, red);
    }
    __syncthreads();  // the next group reuses the tables and the reduction slots
  }
}

// ---- pass A: p_new = y + beta p_old; q = A p_new; partial p_new^T q -------------------
template <int DIM, int QPB, typename TY>
__global__ __launch_bounds__(kThreads) void k_pass_a(StencilGeom g, int64_t ld, int B, int chunks,
                                                     const double* coef,
                                                     const TY* __restrict__ y, int64_t y_ld,
                                                     const double* __restrict__ p_old,
                                                     double* __restrict__ p_new,
                                                     const double* __restrict__ beta,
                                                     const int* __restrict__ active,
                                                     double* __restrict__ part) {
  extern __shared__ double dyn[];
  __shared__ double red[4 * QPB];
  const Tile tl = tile_of(chunks);
  const int q0 = tl.q0 * QPB;
  const unsigned mask = load_group<QPB>(g, coef, q0, B, active, dyn);
  if (!mask) return;
  double acc[QPB], be[QPB];
#pragma unroll
  for (int k = 0; k < QPB; ++k) {
    acc[k] = 0.0;
    be[k] = ((mask >> k) & 1u) ? beta[q0 + k] : 0.0;
  }
#pragma unroll
  for (int t = 0; t < 2 * kPH; ++t) {
    const int pos = paired_pos(g, tl.chunk, t);
    if (pos >= 0) {
      Node<DIM> n;
      node_at<DIM>(g, pos, n);
      const uint32_t up = (uint32_t)pos;
#pragma unroll
      for (int k = 0; k < QPB; ++k) {
        if (!((mask >> k) & 1u)) continue;
        const double* cf = dyn + k * g.ct_size;
        // block-uniform row bases, 32-bit byte offsets
        const TY* yb = y + (size_t)(q0 + k) * y_ld;
        const double* po = p_old + (size_t)(q0 + k) * ld;
        const double b_ = be[k];
        const double pp = (double)at_byte(yb, up * (uint32_t)sizeof(TY)) + b_ * at_byte(po, up * 8u);
        double d;
        const double q = apply_at<DIM, double>(
            n, cf, pp,
            [&](int s) {
              return (double)at_byte(yb, (uint32_t)s * (uint32_t)sizeof(TY)) +
                     b_ * at_byte(po, (uint32_t)s * 8u);
            },
            d);
        at_byte(p_new + (size_t)(q0 + k) * ld, up * 8u) = pp;
        acc[k] += pp * q;
      }
    }
  }
  store_partials<QPB>(acc, mask, q0, tl.chunk, chunks, part, red);
}

// ---- pass B: x += alpha p; r_out = r_in - alpha A p; partial ||r_out||^2 ----------------
// r32 (nullable): an FP32 copy of r_out, rows of ld.  XD: the update of x, 0 as above,
// 1 none (deferred to the next iteration), 2 x = (x + a_prev p_prev) + alpha p.
template <int DIM, int QPB, int XD = 0>
__global__ __launch_bounds__(kThreads) void k_pass_b(StencilGeom g, int64_t ld, int B, int chunks,
                                                     const double* coef,
                                                     const double* __restrict__ p,
                                                     double* __restrict__ x,
                                                     const double* r_in, double* r_out,
                                                     const double* __restrict__ alpha,
                                                     const int* __restrict__ active,
                                                     double* __restrict__ part,
                                                     float* __restrict__ r32,
                                                     const double* __restrict__ p_prev,
                                                     const double* __restrict__ a_prev) {
  extern __shared__ double dyn[];
  __shared__ double red[4 * QPB];
  const Tile tl = tile_of(chunks);
  const int q0 = tl.q0 * QPB;
  const unsigned mask = load_group<QPB>(g, coef, q0, B, active, dyn);
  if (!mask) return;
  double acc[QPB], al[QPB], ap[QPB];
#pragma unroll
  for (int k = 0; k < QPB; ++k) {
    acc[k] = 0.0;
    al[k] = ((mask >> k) & 1u) ? alpha[q0 + k] : 0.0;
    ap[k] = (XD == 2 && ((mask >> k) & 1u)) ? a_prev[q0 + k] : 0.0;
  }
#pragma unroll
  for (int t = 0; t < 2 * kPH; ++t) {
    const int pos = paired_pos(g, tl.chunk, t);
    if (pos >= 0) {
      Node<DIM> n;
      node_at<DIM>(g, pos, n);
      const uint32_t bp = (uint32_t)pos * 8u;
#pragma unroll
      for (int k = 0; k < QPB; ++k) {
        if (!((mask >> k) & 1u)) continue;
        const double* cf = dyn + k * g.ct_size;
        // block-uniform row bases, 32-bit byte offsets
        const size_t o = (size_t)(q0 + k) * ld;
        const double* pb = p + o;
        const double pp = at_byte(pb, bp);
        double d;
        const double q = apply_at<DIM, double>(
            n, cf, pp, [&](int s) { return at_byte(pb, (uint32_t)s * 8u); }, d);
        if (XD == 0) at_byte(x + o, bp) += al[k] * pp;
        if (XD == 2)
          at_byte(x + o, bp) = (at_byte(x + o, bp) + ap[k] * at_byte(p_prev + o, bp)) + al[k] * pp;
        const double r = at_byte(r_in + o, bp) - al[k] * q;
        at_byte(r_out + o, bp) = r;
        if (r32) at_byte(r32 + o, (uint32_t)pos * 4u) = (float)r;
        acc[k] += r * r;
      }
    }
  }
  store_partials<QPB>(acc, mask, q0, tl.chunk, chunks, part, red);
}

// A coordinate in [0, hi] with the parity of v (v itself when it is in range), for the
// loads of lanes whose node lies outside the tile or the grid: a node with the parities of
// the wanted one has its colour on every plane, so its storage position lies next to those
// the neighbouring lanes load and costs no extra cache line; its value is never used.
__device__ __forceinline__ int clamp_same_parity(int v, int hi) {
  const int c = v < 0 ? (v & 1) : (v > hi ? hi - ((v - hi) & 1) : v);
  return (c < 0 || c > hi) ? min(max(v, 0), hi) : c;
}

// ---- 3D passes A and B marching along z --------------------------------------------------
// A block owns QPB queries, an in-plane tile of zr rows x zc columns (at most 512 ZN nodes,
// ZN = 2 or 4 per thread) and a slab of planes, which it walks from bottom to top.  The values
// of the current plane (the tile plus one halo row / column on each side) sit in LDS,
// and every thread keeps the values of its own nodes on the planes below and above in
// registers, so each vector element reaches the block once: the in-plane neighbours
// come from LDS and the z neighbours from registers.  The chunked passes above leave
// the z-neighbour reuse to L2, which does not hold it when several queries share a
// block (their traffic between the two uses of a plane exceeds the 4 MB L2 of an XCD).
// Loads run one step ahead: the next plane's own values and halo, and this plane's x
// and r before the barriers.  Arithmetic is that of apply_at, face by face in order.
struct ZTile {
  int zr, zc;        // rows and columns of an in-plane tile
  int rt, ct;        // tiles along y and x
  int slabs, kslab;  // slabs along z and planes per slab
};
constexpr int kZThreads = 512;
constexpr int kZNodes = 2;  // own nodes per thread by default (zr * zc <= 1024); 4 for taller tiles

template <int QPB, int MODE, typename TY, int ZN, int XD = 0, int NB = 1>
__global__ __launch_bounds__(kZThreads) void k_zmarch(StencilGeom g, ZTile zt, int64_t ld, int B,
                                                      const double* coef,
                                                      const TY* __restrict__ y, int64_t y_ld,
                                                      const double* __restrict__ p_in,
                                                      double* __restrict__ p_out,
                                                      double* __restrict__ x,
                                                      const double* r_in, double* r_out,
                                                      const double* __restrict__ scal,
                                                      const int* __restrict__ active,
                                                      double* __restrict__ part, int pstride,
                                                      float* __restrict__ r32,
                                                      const double* __restrict__ p_prev,
                                                      const double* __restrict__ a_prev) {
  // MODE 0 (pass A): v = y + beta p_in, p_out = v, partial v^T A v.
  // MODE 1 (pass B): v = p_in, x += alpha v, r_out = r_in - alpha A v, partial ||r_out||^2,
  // and the FP32 copy r32 of r_out (rows of ld) unless r32 is null.  XD (pass B) is the
  // update of x: 0 as above, 1 none (deferred to the next iteration), 2 the deferred one
  // first, x = (x + a_prev p_prev) + alpha v, the two updates in their original order.
  constexpr int NW = kZThreads / 64;
  extern __shared__ double dyn[];
  __shared__ double red[NW * QPB];
  const int tiles2 = zt.rt * zt.ct;
  const int tiles = tiles2 * zt.slabs;
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int tile = blk % tiles;
  const int q0 = (blk / tiles) * QPB;
  const int slab = tile / tiles2;
  const int rtile = (tile % tiles2) / zt.ct, ctile = tile % zt.ct;
  double* cfs = dyn;
  const int W2 = zt.zc + 2;  // LDS row pitch (halo column on each side)
  const int plane = (zt.zr + 2) * W2;
  // [NB][QPB][zr + 2][zc + 2]: with two buffers, plane k is staged in buffer k % 2,
  // which the block last read two planes before, so one barrier per plane suffices
  double* pl = dyn + QPB * g.ct_size;
  const unsigned mask = load_group<QPB>(g, coef, q0, B, active, cfs);
  if (!mask) return;
  const int j0 = rtile * zt.zr, i0 = ctile * zt.zc;
  const int k0 = slab * zt.kslab;
  const int k1 = min(g.nz, k0 + zt.kslab);
  const int P = g.nxy;

  double sc[QPB], ap[QPB];
#pragma unroll
  for (int q = 0; q < QPB; ++q) {
    sc[q] = ((mask >> q) & 1u) ? scal[q0 + q] : 0.0;
    ap[q] = (XD == 2 && ((mask >> q) & 1u)) ? a_prev[q0 + q] : 0.0;
  }

  // own nodes: in-plane offset m, LDS slot, x/y coefficient bases, boundary bits
  int m_[ZN], slot[ZN], cb[ZN][4], zxy[ZN];
  unsigned inb[ZN];
  bool own[ZN];
#pragma unroll
  for (int s = 0; s < ZN; ++s) {
    const int u = threadIdx.x + s * kZThreads;
    const int jj = u / zt.zc, ii = u - jj * zt.zc;
    const int i = i0 + ii, j = j0 + jj;
    own[s] = u < zt.zr * zt.zc && i < g.nx && j < g.ny;
    const int ic = own[s] ? i : 0, jc = own[s] ? j : 0;
    m_[s] = ic + g.nx * jc;
    slot[s] = (jj + 1) * W2 + ii + 1;
    const uint32_t tx = g.tab[0][ic], ty = g.tab[1][jc];
    const int sx = tx & 0xff, sy = ty & 0xff;
    cb[s][0] = g.ct_off[0] + ((int)((tx >> 8) & 0xff) * g.ct_s1[0] + sy) * g.ct_s2[0];
    cb[s][1] = g.ct_off[0] + ((int)((tx >> 16) & 0xff) * g.ct_s1[0] + sy) * g.ct_s2[0];
    cb[s][2] = g.ct_off[1] + ((int)((ty >> 8) & 0xff) * g.ct_s1[1] + sx) * g.ct_s2[1];
    cb[s][3] = g.ct_off[1] + ((int)((ty >> 16) & 0xff) * g.ct_s1[1] + sx) * g.ct_s2[1];
    zxy[s] = sx * g.ct_s2[2] + sy;
    inb[s] = (ic > 0 ? 1u : 0u) | (ic < g.nx - 1 ? 2u : 0u) | (jc > 0 ? 4u : 0u) |
             (jc < g.ny - 1 ? 8u : 0u);
  }
  // halo cell of this thread (rows j0-1, j0+zr and columns i0-1, i0+zc of the tile)
  int hm, hslot;
  bool hv;
  {
    const int h = threadIdx.x;
    int jj, ii;
    if (h < zt.zc) { jj = -1; ii = h; }
    else if (h < 2 * zt.zc) { jj = zt.zr; ii = h - zt.zc; }
    else if (h < 2 * zt.zc + zt.zr) { jj = h - 2 * zt.zc; ii = -1; }
    else { jj = h - 2 * zt.zc - zt.zr; ii = zt.zc; }
    const int i = i0 + ii, j = j0 + jj;
    hv = h < 2 * (zt.zc + zt.zr) && i >= 0 && i < g.nx && j >= 0 && j < g.ny;
    hm = hv ? i + g.nx * j : 0;
    hslot = (jj + 1) * W2 + ii + 1;
  }

  auto spos = [&](int L) { return (L & 1) ? g.NR + (L >> 1) : (L >> 1); };
  auto live = [&](int q) { return ((mask >> q) & 1u) != 0; };
  // Every load below is unconditional, from a valid address (a clamped query row and,
  // for nodes outside the tile or the grid, position m = 0); values of such lanes are
  // never read (compute skips them and the boundary bits mask absent neighbours).
  // Loads under a branch would each wait for their data before the next one issued.
  // per-query rows as block-uniform bases, read and written at 32-bit byte offsets
  const double* pq[QPB];
  const TY* yq[QPB];
  double* xq[QPB];
  const double* rq[QPB];
  double* oq[QPB];   // p_out (pass A) or r_out (pass B)
  float* sq[QPB];    // r32 (pass B)
  const double* vq[QPB];  // p_prev (pass B, XD = 2)
#pragma unroll
  for (int q = 0; q < QPB; ++q) {
    const size_t b = (size_t)min(q0 + q, B - 1);
    sq[q] = (MODE == 1 && r32) ? r32 + b * ld : nullptr;
    vq[q] = (MODE == 1 && XD == 2) ? p_prev + b * ld : nullptr;
    pq[q] = p_in + b * ld;
    yq[q] = MODE == 0 ? y + b * y_ld : nullptr;
    xq[q] = MODE == 1 ? x + b * ld : nullptr;
    rq[q] = MODE == 1 ? r_in + b * ld : nullptr;
    oq[q] = (MODE == 0 ? p_out : r_out) + b * ld;
  }
  // Pipelining: every load is issued a full step before its use.  At the top of step k
  // the block issues plane k+3 (raw: y and p apart for pass A, combined two steps later),
  // the halo of plane k+1 and, for pass B, x and r of plane k+1; buffers alternate by the
  // parity of k - k0 and the loop is unrolled by two, so they stay in fixed registers
  // (a loop-carried copy of a just-loaded register waits for it).
  struct Raw {
    double p[ZN][QPB];
    TY y[ZN][QPB];
  };
  struct Halo {
    double p[QPB];
    TY y[QPB];
  };
  struct XR {
    double x[ZN][QPB], r[ZN][QPB], v[ZN][QPB];  // v: p_prev (XD = 2)
  };
  auto load_raw = [&](Raw& r, int k) {
#pragma unroll
    for (int s = 0; s < ZN; ++s) {
      const uint32_t pos = (uint32_t)spos(k * P + m_[s]);
#pragma unroll
      for (int q = 0; q < QPB; ++q) {
        r.p[s][q] = at_byte(pq[q], pos * 8u);
        if (MODE == 0) r.y[s][q] = at_byte(yq[q], pos * (uint32_t)sizeof(TY));
      }
    }
  };
  auto combine = [&](double (&v)[ZN][QPB], const Raw& r) {
#pragma unroll
    for (int s = 0; s < ZN; ++s)
#pragma unroll
      for (int q = 0; q < QPB; ++q)
        v[s][q] = MODE == 0 ? (double)r.y[s][q] + sc[q] * r.p[s][q] : r.p[s][q];
  };
  auto load_halo = [&](Halo& h, int k) {
    const uint32_t pos = (uint32_t)spos(k * P + hm);
#pragma unroll
    for (int q = 0; q < QPB; ++q) {
      h.p[q] = at_byte(pq[q], pos * 8u);
      if (MODE == 0) h.y[q] = at_byte(yq[q], pos * (uint32_t)sizeof(TY));
    }
  };
  auto load_xr = [&](XR& t, int k) {
    if (MODE != 1) return;
#pragma unroll
    for (int s = 0; s < ZN; ++s) {
      const uint32_t pos = (uint32_t)spos(k * P + m_[s]);
#pragma unroll
      for (int q = 0; q < QPB; ++q) {
        if (XD != 1) t.x[s][q] = at_byte(xq[q], pos * 8u);
        t.r[s][q] = at_byte(rq[q], pos * 8u);
        if (XD == 2) t.v[s][q] = at_byte(vq[q], pos * 8u);
      }
    }
  };

  // z data of the slab's planes: tangential state and the coefficient-table offsets of
  // the lower and upper z faces
  int* zinfo = reinterpret_cast<int*>(pl + NB * QPB * plane);  // [kslab][3]
  for (int kk = threadIdx.x; kk < k1 - k0; kk += kZThreads) {
    const uint32_t tz = g.tab[2][k0 + kk];
    zinfo[3 * kk] = tz & 0xff;
    zinfo[3 * kk + 1] = g.ct_off[2] + (int)((tz >> 8) & 0xff) * g.ct_s1[2] * g.ct_s2[2];
    zinfo[3 * kk + 2] = g.ct_off[2] + (int)((tz >> 16) & 0xff) * g.ct_s1[2] * g.ct_s2[2];
  }

  const int klast = g.nz - 1;
  // planes k-1, k, k+1 combined; later planes in flight (clamped planes are never used)
  double vb[ZN][QPB], vc[ZN][QPB], vn[ZN][QPB];
  Raw R0, R1;
  Halo H0, H1;
  XR X0, X1;
  {
    Raw t;
    load_raw(t, max(k0 - 1, 0));
    combine(vb, t);
    load_raw(t, k0);
    combine(vc, t);
    load_raw(t, min(k0 + 1, klast));
    combine(vn, t);
  }
  load_raw(R0, min(k0 + 2, klast));
  load_halo(H0, k0);
  load_xr(X0, k0);

  double acc[QPB];
#pragma unroll
  for (int q = 0; q < QPB; ++q) acc[q] = 0.0;

  // one plane; Rk2 holds plane k+2 (raw), Rk3 receives plane k+3; Hk / Xk hold this
  // plane's halo and x, r; Hn / Xn receive the next plane's
  auto step = [&](int k, Raw& Rk2, Raw& Rk3, Halo& Hk, Halo& Hn, XR& Xk, XR& Xn) {
    load_raw(Rk3, min(k + 3, klast));
    load_halo(Hn, min(k + 1, klast));
    load_xr(Xn, min(k + 1, klast));
    double* const pk = NB == 2 ? pl + (k & 1) * QPB * plane : pl;
    if (NB == 1) __syncthreads();  // the previous plane's LDS reads are done
#pragma unroll
    for (int s = 0; s < ZN; ++s)
      if (own[s])
#pragma unroll
        for (int q = 0; q < QPB; ++q) pk[q * plane + slot[s]] = vc[s][q];
    if (hv)
#pragma unroll
      for (int q = 0; q < QPB; ++q)
        pk[q * plane + hslot] = MODE == 0 ? (double)Hk.y[q] + sc[q] * Hk.p[q] : Hk.p[q];
    __syncthreads();  // the plane is staged (and zinfo is written)
    const int sz = zinfo[3 * (k - k0)];
    const int zlo = zinfo[3 * (k - k0) + 1];
    const int zhi = zinfo[3 * (k - k0) + 2];
    const unsigned zb = (k > 0 ? 16u : 0u) | (k < klast ? 32u : 0u);
#pragma unroll
    for (int s = 0; s < ZN; ++s) {
      if (!own[s]) continue;
      const int pos = spos(k * P + m_[s]);
      const unsigned inner = inb[s] | zb;
      const int ci[6] = {cb[s][0] + sz, cb[s][1] + sz, cb[s][2] + sz, cb[s][3] + sz,
                         zlo + zxy[s], zhi + zxy[s]};
#pragma unroll
      for (int q = 0; q < QPB; ++q) {
        if (!live(q)) continue;
        const double* cf = cfs + q * g.ct_size;
        const double* lp = pk + q * plane + slot[s];
        const double vals[6] = {lp[-1], lp[1], lp[-W2], lp[W2], vb[s][q], vn[s][q]};
        double d = 0.0, off = 0.0;
#pragma unroll
        for (int f = 0; f < 6; ++f) {
          const double c = cf[ci[f]];
          d += c;
          off += c * (((inner >> f) & 1u) ? vals[f] : 0.0);
        }
        const double vp = vc[s][q];
        const double Av = d * vp - off;
        const uint32_t o = (uint32_t)pos * 8u;  // the query is live: its row is q0 + q
        if (MODE == 0) {
          __builtin_nontemporal_store(vp, &at_byte(oq[q], o));
          acc[q] += vp * Av;
        } else {
          if (XD == 0) at_byte(xq[q], o) = Xk.x[s][q] + sc[q] * vp;
          if (XD == 2) at_byte(xq[q], o) = (Xk.x[s][q] + ap[q] * Xk.v[s][q]) + sc[q] * vp;
          const double r = Xk.r[s][q] - sc[q] * Av;
          at_byte(oq[q], o) = r;
          if (r32) at_byte(sq[q], (uint32_t)pos * 4u) = (float)r;
          acc[q] += r * r;
        }
      }
    }
#pragma unroll
    for (int s = 0; s < ZN; ++s)
#pragma unroll
      for (int q = 0; q < QPB; ++q) {
        vb[s][q] = vc[s][q];
        vc[s][q] = vn[s][q];
      }
    combine(vn, Rk2);
  };
  for (int k = k0; k < k1; k += 2) {
    step(k, R0, R1, H0, H1, X0, X1);
    if (k + 1 < k1) step(k + 1, R1, R0, H1, H0, X1, X0);
  }
  // partial sums of the block
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < QPB; ++q) {
    const double v = rbk::wave_sum(acc[q]);
    if (lane == 0) red[q * NW + w] = v;
  }
  __syncthreads();
  if (threadIdx.x < QPB && live(threadIdx.x)) {
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < NW; ++i) t += red[threadIdx.x * NW + i];
    part[(size_t)(q0 + threadIdx.x) * pstride + tile] = t;
  }
}

// ---- one colour half-sweep of Gauss-Seidel on A y = rhs ---------------------------------
// For every node of colour `color`: y_p = (rhs_p - sum_nb A_p,nb y_nb) / A_pp with
// A_p,nb = -c_f (the neighbours all have the other colour).  rhs_b = rhs_scale[b] *
// rhs[b*rhs_ld + p].  Partial sums over the updated nodes: y_p rhs_p (part0) and
// y_p rhs2_p (part1).  Arithmetic in TY (the smoother's precision).  The block's QPB
// coefficient tables sit in LDS interleaved by query (entry e of query k at e QPB + k), so
// one wide LDS read gives a face's coefficient for every query; each thread loads all its
// queries' neighbour values before updating them.  RT = float: rhs is the FP32 copy of an
// FP64 right-hand side (the update rounds rhs to TY = float first, so y is the same).
template <int DIM, int QPB, typename TY, bool NT, typename RT = double>
__global__ __launch_bounds__(kThreads) void k_gs_color(StencilGeom g, int color, int B, int chunks,
                                                       const double* coef,
                                                       TY* __restrict__ y, int64_t y_ld,
                                                       const RT* __restrict__ rhs,
                                                       int64_t rhs_ld,
                                                       const double* __restrict__ rhs_scale,
                                                       const double* __restrict__ rhs2,
                                                       int64_t rhs2_ld,
                                                       const int* __restrict__ active,
                                                       double* __restrict__ part0,
                                                       double* __restrict__ part1) {
  extern __shared__ double dyn[];
  TY* cfi = reinterpret_cast<TY*>(dyn);  // [ct_size][QPB]
  __shared__ double red[4 * QPB];
  const Tile tl = tile_of(chunks);
  const int q0 = tl.q0 * QPB;
  unsigned mask = 0;
#pragma unroll
  for (int k = 0; k < QPB; ++k)
    if (q0 + k < B && (!active || active[q0 + k])) mask |= 1u << k;
  if (!mask) return;  // uniform: the whole block leaves
  for (int e = threadIdx.x; e < QPB * g.ct_size; e += blockDim.x) {
    const int k = e % QPB, i = e / QPB;
    cfi[e] = (q0 + k < B) ? (TY)coef[(size_t)(q0 + k) * g.ct_size + i] : TY(0);
  }
  __syncthreads();
  const int lo = color ? g.NR : 0;
  const int hi = color ? g.N : g.NR;
  double a0[QPB], a1[QPB], fsc[QPB];
  // chunks start at lo rounded down to a line (positions below lo left out)
  // per-query rows: block-uniform bases (clamped to an existing query)
  TY* yq[QPB];
  const RT* rq[QPB];
  const double* r2q[QPB];
#pragma unroll
  for (int k = 0; k < QPB; ++k) {
    a0[k] = a1[k] = 0.0;
    fsc[k] = (rhs_scale && ((mask >> k) & 1u)) ? rhs_scale[q0 + k] : 1.0;
    const size_t b = (size_t)min(q0 + k, B - 1);
    yq[k] = y + b * y_ld;
    rq[k] = rhs + b * rhs_ld;
    r2q[k] = rhs2 ? rhs2 + b * rhs2_ld : nullptr;
  }
  const int base = (lo & ~(kAlign - 1)) + tl.chunk * kThreads * kPT;
#pragma unroll
  for (int t = 0; t < kPT; ++t) {
    const int pos = base + t * kThreads + threadIdx.x;
    if (pos >= lo && pos < hi) {
      Node<DIM> n;
      node_at<DIM>(g, pos, n);
      const uint32_t by = (uint32_t)pos * (uint32_t)sizeof(TY), br = (uint32_t)pos * 8u;
      const uint32_t brt = (uint32_t)pos * (uint32_t)sizeof(RT);
      uint32_t bn[2 * DIM];
#pragma unroll
      for (int f = 0; f < 2 * DIM; ++f) bn[f] = (uint32_t)n.nb[f] * (uint32_t)sizeof(TY);
      // every query's loads first (a retired query's values are not loaded and its
      // update is discarded)
      TY nv[QPB][2 * DIM];
      double fr[QPB];
#pragma unroll
      for (int k = 0; k < QPB; ++k) {
        if ((mask >> k) & 1u) {
#pragma unroll
          for (int f = 0; f < 2 * DIM; ++f) nv[k][f] = at_byte(yq[k], bn[f]);
          // NT (a right-hand side per query): rhs is read once and y not again in this
          // sweep, so both bypass L2, leaving it to the neighbour values; a right-hand
          // side shared by the queries stays cached
          fr[k] = NT ? (double)__builtin_nontemporal_load(&at_byte(rq[k], brt))
                     : (double)at_byte(rq[k], brt);
        } else {
#pragma unroll
          for (int f = 0; f < 2 * DIM; ++f) nv[k][f] = TY(0);
          fr[k] = 0.0;
        }
      }
      TY d[QPB], off[QPB];
#pragma unroll
      for (int k = 0; k < QPB; ++k) d[k] = off[k] = TY(0);
#pragma unroll
      for (int f = 0; f < 2 * DIM; ++f) {
        const TY* cp = cfi + n.ci[f] * QPB;
        const bool in = (n.inner >> f) & 1u;
#pragma unroll
        for (int k = 0; k < QPB; ++k) {
          const TY c = cp[k];
          d[k] += c;
          off[k] += c * (in ? nv[k][f] : TY(0));
        }
      }
#pragma unroll
      for (int k = 0; k < QPB; ++k) {
        if (!((mask >> k) & 1u)) continue;
        const double fp = fsc[k] * fr[k];
        const TY v = gs_div<TY>((TY)fp + off[k], d[k]);
        if (NT)
          __builtin_nontemporal_store(v, &at_byte(yq[k], by));
        else
          at_byte(yq[k], by) = v;
        if (part0) {  // sweeps that leave the class final only (a uniform branch)
          a0[k] += (double)v * fp;
          if (rhs2) a1[k] += (double)v * at_byte(r2q[k], br);
        }
      }
    }
  }
  if (part0) store_partials<QPB>(a0, mask, q0, tl.chunk, chunks, part0, red);
  if (part1) {
    __syncthreads();
    store_partials<QPB>(a1, mask, q0, tl.chunk, chunks, part1, red);
  }
}

// ---- one colour half-sweep marching along z (3D) ----------------------------------------
// Same update and partial sums as k_gs_color, for the nodes of colour `color`.  A block
// owns QPB queries, an in-plane tile of zr rows x zc columns (zc even) and a slab of
// planes.  A thread owns kGsPairs x-adjacent pairs of columns (i0 + 2u, i0 + 2u + 1), in
// rows kGsRowStep apart: on every plane one node of a pair has the swept colour (it is
// updated) and the other the opposite colour (its y is a neighbour value), and they swap
// from plane to plane.  The opposite-colour values of the current plane go to LDS for
// the in-plane neighbours; the z neighbours of an updated node are the opposite-colour
// values of its own column on the planes below and above, which this thread loaded as
// the other node of the pair there, so they stay in registers.  Loads are issued ahead
// as in the marching passes: the neighbour values of plane k+3 (two steps ahead), the
// halo, rhs (and rhs2) of plane k+1.  Partial sums go to part[b * tiles + tile].
constexpr int kGsPairs = 2;  // pairs per thread by default: tiles of up to 2 * 512 / (zc / 2)
                             // rows; 4 for tiles twice as tall
template <int QPB, typename TY, bool FLEX, typename RT = double, int NP = kGsPairs>
__global__ __launch_bounds__(kZThreads) void k_gs_zmarch(StencilGeom g, ZTile zt, int color,
                                                         int B, const double* coef,
                                                         TY* __restrict__ y, int64_t y_ld,
                                                         const RT* __restrict__ rhs,
                                                         int64_t rhs_ld,
                                                         const double* __restrict__ rhs_scale,
                                                         const double* __restrict__ rhs2,
                                                         int64_t rhs2_ld,
                                                         const int* __restrict__ active,
                                                         double* __restrict__ part0,
                                                         double* __restrict__ part1,
                                                         int nbuf) {
  constexpr int NW = kZThreads / 64;
  extern __shared__ double dyn[];
  __shared__ double red[NW * QPB];
  const int tiles2 = zt.rt * zt.ct;
  const int tiles = tiles2 * zt.slabs;
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int tile = blk % tiles;
  const int q0 = (blk / tiles) * QPB;
  const int slab = tile / tiles2;
  const int rtile = (tile % tiles2) / zt.ct, ctile = tile % zt.ct;
  TY* cfs = reinterpret_cast<TY*>(dyn);
  const int W2 = zt.zc + 2;  // LDS row pitch (halo column on each side)
  const int plane = (zt.zr + 2) * W2;
  // [nbuf][QPB][zr + 2][zc + 2]: with two buffers, plane k is staged in buffer k % 2,
  // which the block last read two planes before, so one barrier per plane suffices
  TY* pl = cfs + QPB * g.ct_size;
  const unsigned mask = load_group<QPB, TY>(g, coef, q0, B, active, cfs);
  if (!mask) return;
  const int j0 = rtile * zt.zr, i0 = ctile * zt.zc;  // i0 is even
  const int k0 = slab * zt.kslab;
  const int k1 = min(g.nz, k0 + zt.kslab);
  const int P = g.nxy;
  const int klast = g.nz - 1;

  double fsc[QPB];
#pragma unroll
  for (int q = 0; q < QPB; ++q)
    fsc[q] = (rhs_scale && ((mask >> q) & 1u)) ? rhs_scale[q0 + q] : 1.0;

  // the pairs of columns of this thread: offsets, LDS slots, coefficient bases, boundary
  const int pairs = zt.zc >> 1;
  const int rstep = kZThreads / pairs;  // rows between a thread's pairs
  const int pu = threadIdx.x % pairs;
  // a node outside the tile or the grid is loaded from one of its colour inside them
  const int jlast = min(j0 + zt.zr, g.ny) - 1;  // last row of the tile inside the grid
  // lm0 / lm1: in-plane offsets the two columns of a pair load from (two arrays, not one
  // indexed by the plane's parity, which the compiler kept in scratch memory)
  int j[NP], lm0[NP], lm1[NP], slot[NP][2], cb[NP][2][4], zxy[NP][2];
  unsigned inb[NP][2];
  bool own[NP][2];
#pragma unroll
  for (int a = 0; a < NP; ++a) {
    const int jj = threadIdx.x / pairs + a * rstep;
    j[a] = j0 + jj;
    // threads past rstep * pairs own nothing (their rows belong to the next pair set)
    const bool rowok = (int)threadIdx.x < rstep * pairs && jj < zt.zr && j[a] < g.ny;
    const int jc = rowok ? j[a] : 0;
    const int jl = rowok ? j[a] : clamp_same_parity(j[a], jlast);
#pragma unroll
    for (int c2 = 0; c2 < 2; ++c2) {
      const int i = i0 + 2 * pu + c2;
      own[a][c2] = rowok && i < g.nx;
      const int ic = own[a][c2] ? i : 0;
      (c2 ? lm1[a] : lm0[a]) = clamp_same_parity(i, g.nx - 1) + g.nx * jl;
      slot[a][c2] = (jj + 1) * W2 + 2 * pu + c2 + 1;
      const uint32_t tx = g.tab[0][ic], ty = g.tab[1][jc];
      const int sx = tx & 0xff, sy = ty & 0xff;
      cb[a][c2][0] = g.ct_off[0] + ((int)((tx >> 8) & 0xff) * g.ct_s1[0] + sy) * g.ct_s2[0];
      cb[a][c2][1] = g.ct_off[0] + ((int)((tx >> 16) & 0xff) * g.ct_s1[0] + sy) * g.ct_s2[0];
      cb[a][c2][2] = g.ct_off[1] + ((int)((ty >> 8) & 0xff) * g.ct_s1[1] + sx) * g.ct_s2[1];
      cb[a][c2][3] = g.ct_off[1] + ((int)((ty >> 16) & 0xff) * g.ct_s1[1] + sx) * g.ct_s2[1];
      zxy[a][c2] = sx * g.ct_s2[2] + sy;
      inb[a][c2] = (ic > 0 ? 1u : 0u) | (ic < g.nx - 1 ? 2u : 0u) | (jc > 0 ? 4u : 0u) |
                   (jc < g.ny - 1 ? 8u : 0u);
    }
  }
  // the column of pair a updated on plane k (the colour of node (i, j, k) is the parity
  // of i + j + k, and i0 + 2u is even); the other one holds the neighbour value
  auto ucol = [&](int a, int k) { return (j[a] + k + color) & 1; };
  // Halo (rows j0-1, j0+zr and columns i0-1, i0+zc of the tile): thread h covers two
  // adjacent cells (two columns of a halo row, or two rows of a halo column), which have
  // opposite colours; on each plane only the one of the colour opposite to the swept one
  // is a neighbour value, and the thread loads that one.
  int hmc[2], hsl[2], hpar;
  bool hvc[2];
  {
    const int h = threadIdx.x;
    const int hr = zt.zc >> 1, hc = (zt.zr + 1) >> 1;  // cell pairs per halo row / column
    int hj[2], hi[2];
    bool col = false, any = true;
    if (h < hr) {
      hj[0] = hj[1] = -1;
      hi[0] = 2 * h;
    } else if (h < 2 * hr) {
      hj[0] = hj[1] = zt.zr;
      hi[0] = 2 * (h - hr);
    } else if (h < 2 * hr + hc) {
      col = true;
      hi[0] = hi[1] = -1;
      hj[0] = 2 * (h - 2 * hr);
    } else if (h < 2 * hr + 2 * hc) {
      col = true;
      hi[0] = hi[1] = zt.zc;
      hj[0] = 2 * (h - 2 * hr - hc);
    } else {
      any = false;
      hj[0] = hj[1] = 0;
      hi[0] = 0;
    }
    if (col) hj[1] = hj[0] + 1; else hi[1] = hi[0] + 1;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int i = i0 + hi[c], jh = j0 + hj[c];
      hvc[c] = any && i >= 0 && i < g.nx && jh >= 0 && jh < g.ny && (!col || hj[c] < zt.zr);
      hmc[c] = clamp_same_parity(i, g.nx - 1) + g.nx * clamp_same_parity(jh, g.ny - 1);
      hsl[c] = (hj[c] + 1) * W2 + hi[c] + 1;
    }
    hpar = (i0 + hi[0] + j0 + hj[0]) & 1;  // colour of cell 0 on plane 0
  }
  // the halo cell of the opposite colour on plane k
  auto hsel = [&](int k) { return ((hpar + k) & 1) == (color ^ 1) ? 0 : 1; };

  auto spos = [&](int L) { return (L & 1) ? g.NR + (L >> 1) : (L >> 1); };
  auto live = [&](int q) { return ((mask >> q) & 1u) != 0; };
  // Every load is unconditional, from a valid address (clamped query row; position
  // m = 0 for columns outside the tile or the grid, whose values are never read).
  size_t rowy[QPB], rowr[QPB], rowr2[QPB];
#pragma unroll
  for (int q = 0; q < QPB; ++q) {
    const int b = min(q0 + q, B - 1);
    rowy[q] = (size_t)b * y_ld;
    rowr[q] = (size_t)b * rhs_ld;
    rowr2[q] = FLEX ? (size_t)b * rhs2_ld : 0;
  }
  struct Raw {
    TY v[NP][QPB];
  };
  struct Halo {
    TY v[QPB];
  };
  struct Rhs {
    RT r[NP][QPB];
    double r2[NP][QPB];
  };
  // neighbour values of this thread's column pairs on plane k
  auto load_raw = [&](Raw& t, int k) {
#pragma unroll
    for (int a = 0; a < NP; ++a) {
      const int pos = spos(k * P + (ucol(a, k) ? lm0[a] : lm1[a]));
#pragma unroll
      for (int q = 0; q < QPB; ++q) t.v[a][q] = y[rowy[q] + pos];
    }
  };
  auto load_halo = [&](Halo& t, int k) {
    const int pos = spos(k * P + (hsel(k) ? hmc[1] : hmc[0]));
#pragma unroll
    for (int q = 0; q < QPB; ++q) t.v[q] = y[rowy[q] + pos];
  };
  // right-hand side(s) at the nodes updated on plane k
  auto load_rhs = [&](Rhs& t, int k) {
#pragma unroll
    for (int a = 0; a < NP; ++a) {
      const int pos = spos(k * P + (ucol(a, k) ? lm1[a] : lm0[a]));
#pragma unroll
      for (int q = 0; q < QPB; ++q) {
        t.r[a][q] = rhs[rowr[q] + pos];
        if (FLEX) t.r2[a][q] = rhs2[rowr2[q] + pos];
      }
    }
  };

  int* zinfo = reinterpret_cast<int*>(pl + nbuf * QPB * plane);  // [kslab][3]
  for (int kk = threadIdx.x; kk < k1 - k0; kk += kZThreads) {
    const uint32_t tz = g.tab[2][k0 + kk];
    zinfo[3 * kk] = tz & 0xff;
    zinfo[3 * kk + 1] = g.ct_off[2] + (int)((tz >> 8) & 0xff) * g.ct_s1[2] * g.ct_s2[2];
    zinfo[3 * kk + 2] = g.ct_off[2] + (int)((tz >> 16) & 0xff) * g.ct_s1[2] * g.ct_s2[2];
  }

  // neighbour values of planes k-1, k, k+1; plane k+2 in R0, later planes in flight
  Raw vb, vc, vn, R0, R1;
  Halo H0, H1;
  Rhs X0, X1;
  load_raw(vb, max(k0 - 1, 0));
  load_raw(vc, k0);
  load_raw(vn, min(k0 + 1, klast));
  load_raw(R0, min(k0 + 2, klast));
  load_halo(H0, k0);
  load_rhs(X0, k0);

  double a0[QPB], a1[QPB];
#pragma unroll
  for (int q = 0; q < QPB; ++q) a0[q] = a1[q] = 0.0;

  auto step = [&](int k, Raw& Rk2, Raw& Rk3, Halo& Hk, Halo& Hn, Rhs& Xk, Rhs& Xn) {
    load_raw(Rk3, min(k + 3, klast));
    load_halo(Hn, min(k + 1, klast));
    load_rhs(Xn, min(k + 1, klast));
    TY* const pk = pl + (nbuf == 2 ? (k & 1) * QPB * plane : 0);
    if (nbuf == 1) __syncthreads();  // the previous plane's LDS reads are done
#pragma unroll
    for (int a = 0; a < NP; ++a) {
      const int cu = ucol(a, k);
      if (cu ? own[a][0] : own[a][1]) {
        const int ss = cu ? slot[a][0] : slot[a][1];
#pragma unroll
        for (int q = 0; q < QPB; ++q) pk[q * plane + ss] = vc.v[a][q];
      }
    }
    {
      const int hs = hsel(k);
      if (hs ? hvc[1] : hvc[0])
#pragma unroll
        for (int q = 0; q < QPB; ++q) pk[q * plane + (hs ? hsl[1] : hsl[0])] = Hk.v[q];
    }
    __syncthreads();  // the plane is staged (and zinfo is written)
    const int sz = zinfo[3 * (k - k0)];
    const int zlo = zinfo[3 * (k - k0) + 1];
    const int zhi = zinfo[3 * (k - k0) + 2];
    const unsigned zb = (k > 0 ? 16u : 0u) | (k < klast ? 32u : 0u);
#pragma unroll
    for (int a = 0; a < NP; ++a) {
      const int cu = ucol(a, k);
      if (!(cu ? own[a][1] : own[a][0])) continue;
      const int pos = spos(k * P + (cu ? lm1[a] : lm0[a]));  // an own node
      const unsigned inner = (cu ? inb[a][1] : inb[a][0]) | zb;
      const int su = cu ? slot[a][1] : slot[a][0];
      const int zx = cu ? zxy[a][1] : zxy[a][0];
      const int ci[6] = {(cu ? cb[a][1][0] : cb[a][0][0]) + sz,
                         (cu ? cb[a][1][1] : cb[a][0][1]) + sz,
                         (cu ? cb[a][1][2] : cb[a][0][2]) + sz,
                         (cu ? cb[a][1][3] : cb[a][0][3]) + sz, zlo + zx, zhi + zx};
#pragma unroll
      for (int q = 0; q < QPB; ++q) {
        if (!live(q)) continue;
        const TY* cf = cfs + q * g.ct_size;
        const TY* lp = pk + q * plane + su;
        const TY nv[6] = {lp[-1], lp[1], lp[-W2], lp[W2], vb.v[a][q], vn.v[a][q]};
        TY d = TY(0), off = TY(0);
#pragma unroll
        for (int f = 0; f < 6; ++f) {
          const TY c = cf[ci[f]];
          d += c;
          off += c * (((inner >> f) & 1u) ? nv[f] : TY(0));
        }
        const double fp = fsc[q] * (double)Xk.r[a][q];
        const TY v = gs_div<TY>((TY)fp + off, d);
        y[(size_t)(q0 + q) * y_ld + pos] = v;
        if (part0) {  // sweeps that leave the class final only (a uniform branch)
          a0[q] += (double)v * fp;
          if (FLEX) a1[q] += (double)v * Xk.r2[a][q];
        }
      }
    }
    vb = vc;
    vc = vn;
    vn = Rk2;
  };
  for (int k = k0; k < k1; k += 2) {
    step(k, R0, R1, H0, H1, X0, X1);
    if (k + 1 < k1) step(k + 1, R1, R0, H1, H0, X1, X0);
  }
  // partial sums of the block
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  auto store = [&](const double (&acc)[QPB], double* part) {
    __syncthreads();  // red is free
#pragma unroll
    for (int q = 0; q < QPB; ++q) {
      const double v = rbk::wave_sum(acc[q]);
      if (lane == 0) red[q * NW + w] = v;
    }
    __syncthreads();
    if (threadIdx.x < QPB && live(threadIdx.x)) {
      double t = 0.0;
#pragma unroll
      for (int i = 0; i < NW; ++i) t += red[threadIdx.x * NW + i];
      part[(size_t)(q0 + threadIdx.x) * tiles + tile] = t;
    }
  };
  if (part0) store(a0, part0);
  if (FLEX && part1) store(a1, part1);
}

// ---- one forward red-black sweep, both colours in one walk along z (3D, nx <= 255) ------
// y = S(A, rhs, z) for a start z that is zero on the red nodes: red on plane k from z's
// black values, then black on plane k-1 from the new red values of planes k-2 .. k.  z's
// black values come from zs (its black half), which nothing writes during the sweep, and
// each node of y is written once, by the block that owns it: the red values a block's
// black updates need from outside its tile (the halo rows, and the planes just outside
// its slab) it recomputes itself.  So no block reads what another block writes.  The
// update is k_gs_color's, face by face in the same order and precision: y equals the two
// colour sweeps' y bit for bit.
// A block owns QPB queries, rows j0 .. j0+zr-1 of every plane (whole rows) and a slab of
// planes.  LDS holds per query three planes of z's black values (rows j0-2 .. j0+zr+1)
// and three planes of new red values (rows j0-1 .. j0+zr), one slot per column pair
// (2u, 2u+1) of a row, which holds the pair's node of the stored colour.  A row's nodes of
// one colour are consecutive storage positions, so every load of a plane is contiguous.
// Loads run one step ahead (z's next-but-one plane, the right-hand sides of the next step).
// Partial sums of y^T rhs (and y^T rhs2) go to part[b * tiles + tile].
constexpr int kFusedSlots = 3;  // slots (row, pair) per thread: (zr + 4) * pairs <= 1536

template <int QPB, typename TY, bool FLEX>
__global__ __launch_bounds__(kZThreads) void k_gs_fused(StencilGeom g, ZTile zt, int B,
                                                        const double* coef,
                                                        const TY* __restrict__ zs,
                                                        TY* __restrict__ y, int64_t y_ld,
                                                        const double* __restrict__ rhs,
                                                        int64_t rhs_ld,
                                                        const double* __restrict__ rhs2,
                                                        int64_t rhs2_ld,
                                                        const int* __restrict__ active,
                                                        double* __restrict__ part0,
                                                        double* __restrict__ part1) {
  constexpr int NW = kZThreads / 64;
  constexpr int NS = kFusedSlots;
  extern __shared__ double dyn[];
  __shared__ double red[NW * QPB];
  const int tiles = zt.rt * zt.slabs;
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int tile = blk % tiles;
  const int q0 = (blk / tiles) * QPB;
  const int slab = tile / zt.rt, rtile = tile % zt.rt;
  const int PR = (g.nx + 1) >> 1;  // column pairs per row
  const int ZR2 = zt.zr + 2, ZR4 = zt.zr + 4;
  const int zpl = ZR4 * PR, rpl = ZR2 * PR;  // slots of one LDS plane
  const int qst = 3 * (zpl + rpl);           // LDS per query
  TY* cfs = reinterpret_cast<TY*>(dyn);
  TY* lz = cfs + QPB * g.ct_size;  // [QPB][3][ZR4][PR] z's black values
  TY* lr = lz + 3 * zpl;           // [QPB][3][ZR2][PR] new red values (offset by query)
  const unsigned mask = load_group<QPB, TY>(g, coef, q0, B, active, cfs);
  if (!mask) return;
  const int j0 = rtile * zt.zr;
  const int k0 = slab * zt.kslab;
  const int k1 = min(g.nz, k0 + zt.kslab);
  const int kfirst = max(k0 - 1, 0);
  const int nzm = g.nz - 1;
  int* zinfo = reinterpret_cast<int*>(cfs + QPB * g.ct_size + QPB * qst);  // [k - kfirst][3]
  for (int kk = threadIdx.x; kk <= k1 - kfirst && kfirst + kk <= nzm; kk += kZThreads) {
    const uint32_t tz = g.tab[2][kfirst + kk];
    zinfo[3 * kk] = tz & 0xff;
    zinfo[3 * kk + 1] = g.ct_off[2] + (int)((tz >> 8) & 0xff) * g.ct_s1[2] * g.ct_s2[2];
    zinfo[3 * kk + 2] = g.ct_off[2] + (int)((tz >> 16) & 0xff) * g.ct_s1[2] * g.ct_s2[2];
  }
  auto live = [&](int q) { return ((mask >> q) & 1u) != 0; };
  // storage position of the node of pair u in row j of plane k with colour c (0 red)
  auto spos = [&](int j, int k, int u, int c) {
    const int rb = k * g.nxy + j * g.nx, par = (j + k) & 1;
    return c ? g.NR + ((rb - par) >> 1) + u : ((rb + par) >> 1) + u;
  };
  // the node of colour c in pair u of row j, plane k: column 2u + ((j + k + c) & 1)
  auto col = [&](int j, int k, int u, int c) { return 2 * u + ((j + k + c) & 1); };

  // slots of this thread: s = threadIdx.x + m * kZThreads is (window row s / PR, pair
  // s % PR); the window of the red updates starts at row j0 - 1, that of the staged z
  // values at row j0 - 2
  int wr[NS], su[NS];
  int cb[NS][2][4], zxy[NS][2];
  unsigned inb[NS][2];
  bool cex[NS][2];
#pragma unroll
  for (int m = 0; m < NS; ++m) {
    const int sl = threadIdx.x + m * kZThreads;
    wr[m] = sl / PR;
    su[m] = sl - wr[m] * PR;
    const int j = j0 - 1 + wr[m];
    const bool rowok = wr[m] < ZR2 && j >= 0 && j < g.ny;
    const int jc = rowok ? j : 0;
#pragma unroll
    for (int c2 = 0; c2 < 2; ++c2) {
      const int i = 2 * su[m] + c2;
      cex[m][c2] = rowok && i < g.nx;
      const int ic = cex[m][c2] ? i : 0;
      const uint32_t tx = g.tab[0][ic], ty = g.tab[1][jc];
      const int sx = tx & 0xff, sy = ty & 0xff;
      cb[m][c2][0] = g.ct_off[0] + ((int)((tx >> 8) & 0xff) * g.ct_s1[0] + sy) * g.ct_s2[0];
      cb[m][c2][1] = g.ct_off[0] + ((int)((tx >> 16) & 0xff) * g.ct_s1[0] + sy) * g.ct_s2[0];
      cb[m][c2][2] = g.ct_off[1] + ((int)((ty >> 8) & 0xff) * g.ct_s1[1] + sx) * g.ct_s2[1];
      cb[m][c2][3] = g.ct_off[1] + ((int)((ty >> 16) & 0xff) * g.ct_s1[1] + sx) * g.ct_s2[1];
      zxy[m][c2] = sx * g.ct_s2[2] + sy;
      inb[m][c2] = (ic > 0 ? 1u : 0u) | (ic < g.nx - 1 ? 2u : 0u) | (jc > 0 ? 4u : 0u) |
                   (jc < g.ny - 1 ? 8u : 0u);
    }
  }
  size_t rowy[QPB], rowr[QPB], rowr2[QPB];
#pragma unroll
  for (int q = 0; q < QPB; ++q) {
    const int b = min(q0 + q, B - 1);
    rowy[q] = (size_t)b * y_ld;
    rowr[q] = (size_t)b * rhs_ld;
    rowr2[q] = FLEX ? (size_t)b * rhs2_ld : 0;
  }
  struct ZV {
    TY v[NS][QPB];
  };
  struct RV {
    double r[NS][QPB], r2[NS][QPB];
  };
  // z's black values of plane k, staging rows j0-2 .. j0+zr+1 (every load unconditional,
  // from a valid address: position 0 where the node does not exist)
  auto load_z = [&](ZV& t, int k) __attribute__((always_inline)) {
    const int kc = min(max(k, 0), nzm);
#pragma unroll
    for (int m = 0; m < NS; ++m) {
      const int sl = threadIdx.x + m * kZThreads;
      const int w = sl / PR, u = sl - w * PR, j = j0 - 2 + w;
      const bool ok = k >= 0 && k <= nzm && w < ZR4 && j >= 0 && j < g.ny &&
                      col(j, kc, u, 1) < g.nx;
      const int pos = ok ? spos(j, kc, u, 1) : 0;
#pragma unroll
      for (int q = 0; q < QPB; ++q) t.v[m][q] = zs[rowy[q] + pos];
    }
  };
  auto store_z = [&](const ZV& t, int k) __attribute__((always_inline)) {
    if (k < 0 || k > nzm) return;
    TY* dst = lz + (k % 3) * zpl;
#pragma unroll
    for (int m = 0; m < NS; ++m) {
      const int sl = threadIdx.x + m * kZThreads;
      if (sl < zpl)
#pragma unroll
        for (int q = 0; q < QPB; ++q) dst[q * qst + sl] = t.v[m][q];
    }
  };
  // right-hand sides at the nodes of colour c of this thread's slots on plane k (red:
  // every window row; black: the tile rows)
  auto load_r = [&](RV& t, int k, int c) __attribute__((always_inline)) {
    const int kc = min(max(k, 0), nzm);
#pragma unroll
    for (int m = 0; m < NS; ++m) {
      const int j = j0 - 1 + wr[m];
      const bool rows = c ? (wr[m] >= 1 && wr[m] <= zt.zr) : true;
      const bool ok = k >= 0 && k <= nzm && rows &&
                      ((col(j, kc, su[m], c) & 1) ? cex[m][1] : cex[m][0]);
      const int pos = ok ? spos(j, kc, su[m], c) : 0;
#pragma unroll
      for (int q = 0; q < QPB; ++q) {
        t.r[m][q] = rhs[rowr[q] + pos];
        if (FLEX) t.r2[m][q] = rhs2[rowr2[q] + pos];
      }
    }
  };

  double a0[QPB], a1[QPB];
#pragma unroll
  for (int q = 0; q < QPB; ++q) a0[q] = a1[q] = 0.0;

  // colour c on plane k of the slots whose window rows lie in [wlo, whi]: neighbours from
  // LDS plane array `nb` (three planes of pitch npl; the slot's row in it is wr + roff),
  // right-hand sides from t; write y and the dots on the tile rows of the slab
  auto update = [&](int k, int c, const TY* nb, int npl, int roff,
                    const RV& t) __attribute__((always_inline)) {
    const int kk = k - kfirst;
    const int sz = zinfo[3 * kk], zlo = zinfo[3 * kk + 1], zhi = zinfo[3 * kk + 2];
    const unsigned zb = (k > 0 ? 16u : 0u) | (k < nzm ? 32u : 0u);
    const TY* p0 = nb + (k % 3) * npl;
    const TY* pm = nb + ((k + 2) % 3) * npl;  // plane k - 1
    const TY* pp = nb + ((k + 1) % 3) * npl;  // plane k + 1
    const bool inslab = k >= k0 && k < k1;
#pragma unroll
    for (int m = 0; m < NS; ++m) {
      const int j = j0 - 1 + wr[m];
      const int c2 = col(j, k, su[m], c) & 1;  // (selects below keep the arrays in registers)
      if (!(c2 ? cex[m][1] : cex[m][0])) continue;
      const bool tilerow = wr[m] >= 1 && wr[m] <= zt.zr;
      if (c && !tilerow) continue;  // black: tile rows only
      const unsigned inner = (c2 ? inb[m][1] : inb[m][0]) | zb;
      const int zx = c2 ? zxy[m][1] : zxy[m][0];
      const int ci[6] = {(c2 ? cb[m][1][0] : cb[m][0][0]) + sz,
                         (c2 ? cb[m][1][1] : cb[m][0][1]) + sz,
                         (c2 ? cb[m][1][2] : cb[m][0][2]) + sz,
                         (c2 ? cb[m][1][3] : cb[m][0][3]) + sz, zlo + zx, zhi + zx};
      const int r0 = (wr[m] + roff) * PR, u = su[m];
      const int ixl = r0 + max(u - 1 + c2, 0), ixh = r0 + u + c2;
      const bool out = inslab && tilerow;
      const int pos = spos(j, k, u, c);
#pragma unroll
      for (int q = 0; q < QPB; ++q) {
        if (!live(q)) continue;
        const TY* cf = cfs + q * g.ct_size;
        const int qo = q * qst;
        const TY nv[6] = {p0[qo + ixl], p0[qo + ixh], p0[qo + r0 - PR + u], p0[qo + r0 + PR + u],
                          pm[qo + r0 + u], pp[qo + r0 + u]};
        TY d = TY(0), off = TY(0);
#pragma unroll
        for (int f = 0; f < 6; ++f) {
          const TY cc = cf[ci[f]];
          d += cc;
          off += cc * (((inner >> f) & 1u) ? nv[f] : TY(0));
        }
        const double fp = t.r[m][q];
        const TY v = gs_div<TY>((TY)fp + off, d);
        if (!c) lr[qo + (k % 3) * rpl + wr[m] * PR + u] = v;
        if (out) {
          y[rowy[q] + pos] = v;
          a0[q] += (double)v * fp;
          if (FLEX) a1[q] += (double)v * t.r2[m][q];
        }
      }
    }
  };

  // z planes kfirst - 1 and kfirst into LDS; plane kfirst + 1 and the right-hand sides of
  // the first step in flight
  ZV Za, Zb;
  RV Ra, Rb, Ba, Bb;
  load_z(Za, kfirst - 1);
  store_z(Za, kfirst - 1);
  load_z(Za, kfirst);
  store_z(Za, kfirst);
  load_z(Za, kfirst + 1);
  load_r(Ra, kfirst, 0);
  load_r(Ba, kfirst - 1, 1);
  auto step = [&](int k, ZV& Zn, ZV& Zn2, RV& Rn, RV& Rn2, RV& Bn,
                  RV& Bn2) __attribute__((always_inline)) {
    // Zn = z plane k + 1, Rn = red right-hand sides of plane k, Bn = black ones of plane
    // k - 1, all loaded a step ahead; the next step's are issued before the barriers
    store_z(Zn, k + 1);
    load_z(Zn2, k + 2);
    load_r(Rn2, k + 1, 0);
    load_r(Bn2, k, 1);
    __syncthreads();  // z plane k + 1 (and zinfo) visible; the black updates of k - 2 done
    if (k <= nzm) update(k, 0, lz, zpl, 1, Rn);
    __syncthreads();  // red plane k visible
    if (k - 1 >= k0) update(k - 1, 1, lr, rpl, 0, Bn);
  };
  for (int k = kfirst; k <= k1; k += 2) {
    step(k, Za, Zb, Ra, Rb, Ba, Bb);
    if (k + 1 <= k1) step(k + 1, Zb, Za, Rb, Ra, Bb, Ba);
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  auto store = [&](const double (&acc)[QPB], double* part) {
    __syncthreads();  // red is free
#pragma unroll
    for (int q = 0; q < QPB; ++q) {
      const double v = rbk::wave_sum(acc[q]);
      if (lane == 0) red[q * NW + w] = v;
    }
    __syncthreads();
    if (threadIdx.x < QPB && live(threadIdx.x)) {
      double t = 0.0;
#pragma unroll
      for (int i = 0; i < NW; ++i) t += red[threadIdx.x * NW + i];
      part[(size_t)(q0 + threadIdx.x) * tiles + tile] = t;
    }
  };
  if (part0) store(a0, part0);
  if (FLEX && part1) store(a1, part1);
}

// ---- damped Jacobi: y = z + omega D^-1 (rhs - A z), partial y^T rhs (and y^T rhs2) ------
template <int DIM, int QPB, typename TY>
__global__ __launch_bounds__(kThreads) void k_jacobi(StencilGeom g, int B, int chunks,
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
  extern __shared__ double dyn[];
  TY* cfs = reinterpret_cast<TY*>(dyn);
  __shared__ double red[4 * QPB];
  const Tile tl = tile_of(chunks);
  const int q0 = tl.q0 * QPB;
  const unsigned mask = load_group<QPB>(g, coef, q0, B, active, cfs);
  if (!mask) return;
  double a0[QPB], a1[QPB];
#pragma unroll
  for (int k = 0; k < QPB; ++k) a0[k] = a1[k] = 0.0;
#pragma unroll
  for (int t = 0; t < 2 * kPH; ++t) {
    const int pos = paired_pos(g, tl.chunk, t);
    if (pos >= 0) {
      Node<DIM> n;
      node_at<DIM>(g, pos, n);
#pragma unroll
      for (int k = 0; k < QPB; ++k) {
        if (!((mask >> k) & 1u)) continue;
        const TY* cf = cfs + k * g.ct_size;
        const TY* zb = z + (size_t)(q0 + k) * y_ld;
        TY d;
        const TY Az = apply_at<DIM, TY>(n, cf, zb[pos], [&](int s) { return zb[s]; }, d);
        const double fp = rhs[(size_t)(q0 + k) * rhs_ld + pos];
        const TY v = zb[pos] + (TY)omega * (((TY)fp - Az) / d);
        y[(size_t)(q0 + k) * y_ld + pos] = v;
        a0[k] += (double)v * fp;
        if (rhs2) a1[k] += (double)v * rhs2[(size_t)(q0 + k) * rhs2_ld + pos];
      }
    }
  }
  if (part0) store_partials<QPB>(a0, mask, q0, tl.chunk, chunks, part0, red);
  if (part1) {
    __syncthreads();
    store_partials<QPB>(a1, mask, q0, tl.chunk, chunks, part1, red);
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
  if (p.g.csr) return csr_to_storage(p.g.N, p.perm.as<int>(), B, nat, nat_ld, sto, sto_ld, s);
  hipLaunchKernelGGL(k_to_storage, conv_grid(p.g.N, B), dim3(256), 0, s, p.g.N, p.g.NR, nat,
                     nat_ld, sto, sto_ld);
}
void launch_from_storage(const rb_problem& p, int B, const double* sto, int64_t sto_ld,
                         double* nat, int64_t nat_ld, hipStream_t s) {
  if (p.g.csr)
    return csr_from_storage(p.g.N, p.perm.as<int>(), B, sto, sto_ld, nat, nat_ld, s);
  hipLaunchKernelGGL(k_from_storage, conv_grid(p.g.N, B), dim3(256), 0, s, p.g.N, p.g.NR, sto,
                     sto_ld, nat, nat_ld);
}

// ---- launchers -----------------------------------------------------------------------
int stencil_chunks(int count) { return (count + kThreads * kPT - 1) / (kThreads * kPT); }
int stencil_chunks_all(int N) {
  const int NR = (N + 1) / 2;
  const int CH = kThreads * kPH;
  // red [0, NR) and black [NR rounded down to kAlign, N) (paired_pos)
  return std::max((NR + CH - 1) / CH, (N - (NR & ~(kAlign - 1)) + CH - 1) / CH);
}
int stencil_sweep_chunks(int lo, int hi) { return stencil_chunks(hi - (lo & ~(kAlign - 1))); }

static thread_local TuneConfig t_tiles;
void set_stencil_tiles(const TuneConfig& c) { t_tiles = c; }
TuneConfig stencil_tiles() { return t_tiles; }

// queries per block: up to `cap` while the group's tables stay within 16 KB of LDS.
// Measured on the 127^3 workload (B = 256): pass A (two arrays read at the
// neighbours) is fastest with 1-2 queries per block, the one-colour sweeps with 4.
static int pick_qpb(const StencilGeom& g, int B, int tsize, int cap = 4) {
  int q = 1;
  while (q * 2 <= cap && q * 2 <= RB_QPB_MAX) q *= 2;
  while (q > 1 && (q > B || q * g.ct_size * tsize > 16384)) q >>= 1;
  return q;
}

template <typename F>
static void dispatch(int dim, int qpb, F&& f) {
#define RB_Q(D)                                                    \
  switch (qpb) {                                                   \
    case 8: f(std::integral_constant<int, D>{}, std::integral_constant<int, 8>{}); break; \
    case 4: f(std::integral_constant<int, D>{}, std::integral_constant<int, 4>{}); break; \
    case 2: f(std::integral_constant<int, D>{}, std::integral_constant<int, 2>{}); break; \
    default: f(std::integral_constant<int, D>{}, std::integral_constant<int, 1>{}); break; \
  }
  switch (dim) {
    case 1: RB_Q(1) break;
    case 2: RB_Q(2) break;
    default: RB_Q(3) break;
  }
#undef RB_Q
}

static dim3 grid_for(int chunks, int B, int qpb) {
  const long total = (long)chunks * ((B + qpb - 1) / qpb);
  return dim3((unsigned)total);
}

void launch_apply(const StencilGeom& g, int64_t ld, int B, const double* coef, const double* u,
                  double* y, int mode, const double* rhs, int64_t rhs_ld, const double* rhs_scale,
                  const int* flag, double* part, hipStream_t s, double* part2, float* y32) {
  RB_REQUIRE(!y32 || (mode == 1 && !g.csr), RB_EINVAL,
             "FP32 residual copy: mode 1 on stencil grids only");
  if (g.csr)
    return csr_apply(g, ld, B, coef, u, y, mode, rhs, rhs_ld, rhs_scale, flag, part, s, part2);
  const int chunks = stencil_chunks_all(g.N);
  const int qpb = pick_qpb(g, B, 8);
  dispatch(g.dim, qpb, [&](auto D, auto Q) {
    // mode 1 (true residual of the flagged queries) runs every iteration, mostly with
    // no or few flags: one block per chunk visits the groups holding a flag (127^3,
    // B = 256: 35 us per launch without flags and 72 us on average in a solve, against
    // 53 and 111 us with 4 blocks per chunk)
    const int groups = (B + Q.value - 1) / Q.value;
    const int slots = mode == 1 ? (groups + 32 * kApplyMaxGroupWords - 1) /
                                      (32 * kApplyMaxGroupWords)
                                : groups;
    hipLaunchKernelGGL((k_apply<D.value, Q.value>), dim3((unsigned)((long)chunks * slots)),
                       dim3(kThreads), Q.value * g.ct_size * 8, s, g, ld, B, chunks, coef, u, y,
                       mode, rhs, rhs_ld, rhs_scale, flag, part, part2, y32);
  });
}

// Tile of the z-marching passes for `groups` query groups; false if the grid does not
// suit them (not 3D, or more partial sums than the chunked passes produce).
// zn: own nodes per thread (2, or 4 for tiles twice as tall, whose halo rows are a smaller
// share of the rows read).
static bool z_plan(const StencilGeom& g, int groups, ZTile& zt, int zn = kZNodes) {
  if (g.dim != 3) return false;
  // full rows while one thread per halo cell suffices: a tile as wide as the grid has no
  // valid halo columns, so only its two halo rows need threads
  zt.zc = 2 * g.nx <= kZThreads ? g.nx : 128;
  zt.zr = std::min(g.ny, (kZThreads * zn) / zt.zc);
  const int halo = zt.zc == g.nx ? 2 * zt.zc : 2 * (zt.zc + zt.zr);
  if (zt.zr < 1 || halo > kZThreads) return false;
  zt.ct = (g.nx + zt.zc - 1) / zt.zc;
  zt.rt = (g.ny + zt.zr - 1) / zt.zr;
  const int tiles2 = zt.rt * zt.ct;
  const int cap = stencil_chunks_all(g.N);  // partial sums per query the solver holds
  if (tiles2 > cap) return false;
  // about 2048 blocks over the chip, slabs of at least 8 planes
  int slabs = (2048 + groups * tiles2 - 1) / (groups * tiles2);
  slabs = std::max(1, std::min({slabs, g.nz / 8, cap / tiles2}));
  zt.kslab = (g.nz + slabs - 1) / slabs;
  zt.slabs = (g.nz + zt.kslab - 1) / zt.kslab;
  return true;
}

static size_t z_lds(const StencilGeom& g, const ZTile& zt, int qpb, int nbuf = 1) {
  return (size_t)qpb * (g.ct_size + nbuf * (zt.zr + 2) * (zt.zc + 2)) * sizeof(double) +
         (size_t)3 * zt.kslab * sizeof(int);
}

// kind: 1 chunked, 2 z-marching, 0 default: z-marching on 3D batches that give at least
// one block per CU without slabs.  Measured on the 127^3 workload (B = 256, all queries
// active, 2 queries per block): pass A 4.04 ms chunked vs 2.35 ms marching; pass B
// 5.02 ms chunked vs 4.19 ms marching.  Pass B's x and r go through plain loads and
// stores: with non-temporal ones it took 5.22 ms.  Returns the number of partial sums
// per query.
template <int MODE, typename TY>
static int launch_zmarch(const StencilGeom& g, int qpb, int64_t ld, int B, const double* coef,
                         const TY* y, int64_t y_ld, const double* p_in, double* p_out, double* x,
                         const double* r_in, double* r_out, const double* scal,
                         const int* active, double* part, hipStream_t s, int kind,
                         float* r32 = nullptr, int zn = kZNodes, int xd = 0,
                         const double* p_prev = nullptr, const double* a_prev = nullptr) {
  if (kind == 1) return 0;
  qpb = std::min(qpb, 4);
  if (zn != 4 || qpb > 2) zn = kZNodes;  // four nodes per thread: up to two queries per block
  ZTile zt;
  const int groups = (B + qpb - 1) / qpb;
  if (!z_plan(g, groups, zt, zn) || z_lds(g, zt, qpb) > 65536) return 0;
  if (kind == 0 && groups * zt.rt * zt.ct < 256) return 0;
  const int tiles = zt.rt * zt.ct * zt.slabs;
  const int pstride = stencil_chunks_all(g.N);  // row stride of the partial sums
  const dim3 grid((unsigned)(tiles * groups));
  // two plane buffers (one barrier per plane) where they fit in 64 KB: pass B unless the
  // tiles ask for one, pass A when they ask for two (its variants with one buffer need
  // fewer registers)
  const bool two = MODE == 1 ? t_tiles.nb_b != 1 : t_tiles.nb_a == 2;
  const int nbuf = two && z_lds(g, zt, qpb, 2) <= 65536 ? 2 : 1;
  const size_t lds = z_lds(g, zt, qpb, nbuf);
  auto go = [&](auto Q, auto Z) {
    auto run = [&](auto X, auto NBc) {
      hipLaunchKernelGGL((k_zmarch<Q.value, MODE, TY, Z.value, X.value, NBc.value>), grid,
                         dim3(kZThreads), lds, s, g, zt, ld, B, coef, y, y_ld, p_in, p_out, x,
                         r_in, r_out, scal, active, part, pstride, r32, p_prev, a_prev);
    };
    using N1 = std::integral_constant<int, 1>;
    using N2 = std::integral_constant<int, 2>;
    auto by_nb = [&](auto X) { return nbuf == 2 ? run(X, N2{}) : run(X, N1{}); };
    if constexpr (MODE == 1) {
      if (xd == 1) return by_nb(std::integral_constant<int, 1>{});
      if (xd == 2) return by_nb(std::integral_constant<int, 2>{});
    }
    by_nb(std::integral_constant<int, 0>{});
  };
  using Z2 = std::integral_constant<int, kZNodes>;
  using Z4 = std::integral_constant<int, 4>;
  switch (qpb) {
    case 4: go(std::integral_constant<int, 4>{}, Z2{}); break;
    case 2:
      if (zn == 4) go(std::integral_constant<int, 2>{}, Z4{});
      else go(std::integral_constant<int, 2>{}, Z2{});
      break;
    default:
      if (zn == 4) go(std::integral_constant<int, 1>{}, Z4{});
      else go(std::integral_constant<int, 1>{}, Z2{});
      break;
  }
  return tiles;
}

bool zmarch_two_buffers(const StencilGeom& g, int B, int qpb, int zn) {
  qpb = std::min(qpb, 4);
  if (zn != 4 || qpb > 2) zn = kZNodes;
  ZTile zt;
  return z_plan(g, (B + qpb - 1) / qpb, zt, zn) && z_lds(g, zt, qpb, 2) <= 65536;
}

template <typename TY>
int launch_pass_a(const StencilGeom& g, int64_t ld, int B, const double* coef, const TY* y,
                  int64_t y_ld, const double* p_old, double* p_new, const double* beta,
                  const int* active, double* part, hipStream_t s) {
  if (g.csr) return csr_pass_a<TY>(g, ld, B, coef, y, y_ld, p_old, p_new, beta, active, part, s);
  // untuned: 2 queries per block chunked, 1 marching (127^3, B = 256: 2.35 ms vs 2.51 ms
  // with 2)
  const int qpb = pick_qpb(g, B, 8, t_tiles.qpb_a ? t_tiles.qpb_a : 2);
  if (const int t = launch_zmarch<0, TY>(g, t_tiles.qpb_a ? qpb : 1, ld, B, coef, y, y_ld, p_old,
                                         p_new, nullptr, nullptr, nullptr, beta, active, part, s,
                                         t_tiles.kind_a, nullptr,
                                         t_tiles.zn_a ? t_tiles.zn_a : kZNodes))
    return t;
  const int chunks = stencil_chunks_all(g.N);
  dispatch(g.dim, qpb, [&](auto D, auto Q) {
    hipLaunchKernelGGL((k_pass_a<D.value, Q.value, TY>), grid_for(chunks, B, Q.value),
                       dim3(kThreads), Q.value * g.ct_size * 8, s, g, ld, B, chunks, coef, y, y_ld,
                       p_old, p_new, beta, active, part);
  });
  return chunks;
}
template int launch_pass_a<double>(const StencilGeom&, int64_t, int, const double*,
                                   const double*, int64_t, const double*, double*,
                                   const double*, const int*, double*, hipStream_t);
template int launch_pass_a<float>(const StencilGeom&, int64_t, int, const double*, const float*,
                                  int64_t, const double*, double*, const double*, const int*,
                                  double*, hipStream_t);

int launch_pass_b(const StencilGeom& g, int64_t ld, int B, const double* coef, const double* p,
                  double* x, const double* r_in, double* r_out, const double* alpha,
                  const int* active, double* part, hipStream_t s, float* r32, int xd,
                  const double* p_prev, const double* a_prev) {
  RB_REQUIRE(!r32 || !g.csr, RB_EINVAL, "FP32 residual copy: stencil grids only");
  RB_REQUIRE(xd == 0 || !g.csr, RB_EINVAL, "paired updates of x: stencil grids only");
  RB_REQUIRE(xd >= 0 && xd <= 2 && (xd != 2 || (p_prev && a_prev)), RB_EINVAL,
             "bad x update of pass B");
  if (g.csr) return csr_pass_b(g, ld, B, coef, p, x, r_in, r_out, alpha, active, part, s);
  const int qpb = pick_qpb(g, B, 8, t_tiles.qpb_b ? t_tiles.qpb_b : 2);
  if (const int t = launch_zmarch<1, double>(g, qpb, ld, B, coef, nullptr, 0, p, nullptr, x, r_in,
                                             r_out, alpha, active, part, s, t_tiles.kind_b, r32,
                                             t_tiles.zn_b ? t_tiles.zn_b : kZNodes, xd, p_prev,
                                             a_prev))
    return t;
  const int chunks = stencil_chunks_all(g.N);
  dispatch(g.dim, qpb, [&](auto D, auto Q) {
    auto run = [&](auto X) {
      hipLaunchKernelGGL((k_pass_b<D.value, Q.value, X.value>), grid_for(chunks, B, Q.value),
                         dim3(kThreads), Q.value * g.ct_size * 8, s, g, ld, B, chunks, coef, p, x,
                         r_in, r_out, alpha, active, part, r32, p_prev, a_prev);
    };
    if (xd == 1)
      run(std::integral_constant<int, 1>{});
    else if (xd == 2)
      run(std::integral_constant<int, 2>{});
    else
      run(std::integral_constant<int, 0>{});
  });
  return chunks;
}

// Tile of the marching colour sweeps: an even number of columns (pairs per thread), at
// most `cap` tiles per query (the partial sums the solver holds for one colour).
static bool zg_plan(const StencilGeom& g, int groups, int cap, ZTile& zt, int np = kGsPairs) {
  if (g.dim != 3) return false;
  // whole rows up to 255 columns (nx odd: the last column of the last tile is outside),
  // so that no halo column is read: a halo column costs one cache line per row
  zt.zc = std::min(g.nx + 1, 256);
  const int pairs = zt.zc / 2;
  zt.zr = std::min(g.ny, np * (kZThreads / pairs));
  // one thread per pair of halo cells
  if (zt.zr < 1 || 2 * pairs + 2 * ((zt.zr + 1) / 2) > kZThreads) return false;
  zt.ct = (g.nx + zt.zc - 1) / zt.zc;
  zt.rt = (g.ny + zt.zr - 1) / zt.zr;
  const int tiles2 = zt.rt * zt.ct;
  if (tiles2 > cap) return false;
  int slabs = (2048 + groups * tiles2 - 1) / (groups * tiles2);
  slabs = std::max(1, std::min({slabs, g.nz / 8, cap / tiles2}));
  zt.kslab = (g.nz + slabs - 1) / slabs;
  zt.slabs = (g.nz + zt.kslab - 1) / zt.kslab;
  return true;
}

// kind: 1 chunked, 2 marching, 0 default: chunked.  Measured on the 127^3 workload
// (B = 256, FP32): a sweep takes 1.03 ms chunked with 4 queries per block and 1.03-1.08 ms
// marching with 2, 1 or 4 (1.05-1.09 ms with one column pair per thread): a sweep moves
// only 8 B per node per barrier pair of each plane, against pass B's 40.  The autotuner
// tries both.  Returns the number of partial sums per query (0: not run).
template <typename TY, typename RT>
static int launch_gs_zmarch(const StencilGeom& g, int color, int qpb, int B, const double* coef,
                            TY* y, int64_t y_ld, const RT* rhs, int64_t rhs_ld,
                            const double* rhs_scale, const double* rhs2, int64_t rhs2_ld,
                            const int* active, double* part0, double* part1, hipStream_t s,
                            int kind, int np = kGsPairs) {
  if (kind != 2) return 0;
  qpb = std::min(qpb, 4);
  if (np != 4 || qpb > 2) np = kGsPairs;  // four pairs per thread: up to two queries
  ZTile zt;
  const int groups = (B + qpb - 1) / qpb;
  if (!zg_plan(g, groups, stencil_chunks(color ? g.N - g.NR : g.NR), zt, np)) return 0;
  // two plane buffers (one barrier per plane) when they fit in 64 KB, else one
  auto lds_of = [&](int nb) {
    return (size_t)qpb * (g.ct_size + nb * (zt.zr + 2) * (zt.zc + 2)) * sizeof(TY) +
           (size_t)3 * zt.kslab * sizeof(int);
  };
  const int nbuf = lds_of(2) <= 65536 ? 2 : 1;
  const size_t lds = lds_of(nbuf);
  if (lds > 65536) return 0;
  const int tiles = zt.rt * zt.ct * zt.slabs;
  const dim3 grid((unsigned)(tiles * groups));
  auto go = [&](auto Q, auto F, auto NPc) {
    hipLaunchKernelGGL((k_gs_zmarch<Q.value, TY, F.value, RT, NPc.value>), grid, dim3(kZThreads),
                       lds, s, g, zt, color, B, coef, y, y_ld, rhs, rhs_ld, rhs_scale, rhs2,
                       rhs2_ld, active, part0, part1, nbuf);
  };
  using P2 = std::integral_constant<int, kGsPairs>;
  using P4 = std::integral_constant<int, 4>;
  auto by_q = [&](auto F) {
    switch (qpb) {
      case 4: go(std::integral_constant<int, 4>{}, F, P2{}); break;
      case 2:
        if (np == 4) go(std::integral_constant<int, 2>{}, F, P4{});
        else go(std::integral_constant<int, 2>{}, F, P2{});
        break;
      default:
        if (np == 4) go(std::integral_constant<int, 1>{}, F, P4{});
        else go(std::integral_constant<int, 1>{}, F, P2{});
        break;
    }
  };
  if (rhs2)
    by_q(std::true_type{});
  else
    by_q(std::false_type{});
  return tiles;
}

// Tile of the fused sweep: whole rows (nx <= 255), zr <= 16 rows such that the staged
// window of zr + 4 rows fits the threads' slots and the LDS stays within 64 KB; slabs as
// for the marching passes.  lds = dynamic LDS bytes.
static bool zf_plan(const StencilGeom& g, int groups, int cap, int qpb, size_t tysz, ZTile& zt,
                    size_t& lds) {
  if (!gs_fused_supported(g)) return false;
  const int PR = (g.nx + 1) / 2;
  auto lds_of = [&](int zr, int kslab) {
    return (size_t)qpb * (g.ct_size + 3 * (2 * zr + 6) * PR) * tysz +
           (size_t)3 * (kslab + 2) * sizeof(int);
  };
  int zr = std::min({g.ny, 16, kFusedSlots * kZThreads / PR - 4});
  while (zr >= 1 && lds_of(zr, g.nz) > 65536) --zr;
  if (zr < 1) return false;
  zt.zr = zr;
  zt.zc = g.nx;
  zt.ct = 1;
  zt.rt = (g.ny + zr - 1) / zr;
  if (zt.rt > cap) return false;
  int slabs = (2048 + groups * zt.rt - 1) / (groups * zt.rt);
  slabs = std::max(1, std::min({slabs, g.nz / 8, cap / zt.rt}));
  zt.kslab = (g.nz + slabs - 1) / slabs;
  zt.slabs = (g.nz + zt.kslab - 1) / zt.kslab;
  lds = lds_of(zr, zt.kslab);
  return true;
}

bool gs_fused_supported(const StencilGeom& g) {
  return g.dim == 3 && !g.csr && g.C == 2 && g.nx <= 255;
}

template <typename TY>
int launch_gs_fused(const StencilGeom& g, int B, const double* coef, const TY* zs, TY* y,
                    int64_t y_ld, const double* rhs, int64_t rhs_ld, const double* rhs2,
                    int64_t rhs2_ld, const int* active, double* part0, double* part1, int cap,
                    hipStream_t s) {
  // 1 or 2 queries per block (4 would spill registers)
  const int qpb = (t_tiles.qpb_gs ? t_tiles.qpb_gs : 2) >= 2 && B >= 2 ? 2 : 1;
  ZTile zt;
  size_t lds = 0;
  const int groups = (B + qpb - 1) / qpb;
  if (!zf_plan(g, groups, cap, qpb, sizeof(TY), zt, lds)) return 0;
  const int tiles = zt.rt * zt.slabs;
  const dim3 grid((unsigned)(tiles * groups));
  auto go = [&](auto Q, auto F) {
    hipLaunchKernelGGL((k_gs_fused<Q.value, TY, F.value>), grid, dim3(kZThreads), lds, s, g, zt, B,
                       coef, zs, y, y_ld, rhs, rhs_ld, rhs2, rhs2_ld, active, part0, part1);
  };
  auto by_q = [&](auto F) {
    if (qpb == 2)
      go(std::integral_constant<int, 2>{}, F);
    else
      go(std::integral_constant<int, 1>{}, F);
  };
  if (rhs2)
    by_q(std::true_type{});
  else
    by_q(std::false_type{});
  return tiles;
}
template int launch_gs_fused<double>(const StencilGeom&, int, const double*, const double*,
                                     double*, int64_t, const double*, int64_t, const double*,
                                     int64_t, const int*, double*, double*, int, hipStream_t);
template int launch_gs_fused<float>(const StencilGeom&, int, const double*, const float*, float*,
                                    int64_t, const double*, int64_t, const double*, int64_t,
                                    const int*, double*, double*, int, hipStream_t);

template <typename TY, typename RT>
int launch_gs_color(const StencilGeom& g, int color, int B, const double* coef, TY* y,
                    int64_t y_ld, const RT* rhs, int64_t rhs_ld, const double* rhs_scale,
                    const double* rhs2, int64_t rhs2_ld, const int* active, double* part0,
                    double* part1, hipStream_t s) {
  if (g.csr) {
    if constexpr (std::is_same<RT, double>::value) {
      csr_gs_color<TY>(g, color, B, coef, y, y_ld, rhs, rhs_ld, rhs_scale, rhs2, rhs2_ld, active,
                       part0, part1, s);
      return stencil_chunks(g.coff[color + 1] - g.coff[color]);
    } else {
      RB_REQUIRE(false, RB_EINVAL, "FP32 right-hand side: stencil grids only");
    }
  }
  const int qpb = pick_qpb(g, B, (int)sizeof(TY), t_tiles.qpb_gs ? t_tiles.qpb_gs : 4);
  if (const int t = launch_gs_zmarch<TY, RT>(g, color, qpb, B, coef, y, y_ld, rhs, rhs_ld,
                                             rhs_scale, rhs2, rhs2_ld, active, part0, part1, s,
                                             t_tiles.kind_gs,
                                             t_tiles.np_gs ? t_tiles.np_gs : kGsPairs))
    return t;
  const int chunks = color ? stencil_sweep_chunks(g.NR, g.N) : stencil_sweep_chunks(0, g.NR);
  dispatch(g.dim, qpb, [&](auto D, auto Q) {
    const size_t lds = Q.value * g.ct_size * sizeof(TY);
    if (rhs_ld)
      hipLaunchKernelGGL((k_gs_color<D.value, Q.value, TY, true, RT>),
                         grid_for(chunks, B, Q.value), dim3(kThreads), lds, s, g, color, B,
                         chunks, coef, y, y_ld, rhs, rhs_ld, rhs_scale, rhs2, rhs2_ld, active,
                         part0, part1);
    else
      hipLaunchKernelGGL((k_gs_color<D.value, Q.value, TY, false, RT>),
                         grid_for(chunks, B, Q.value), dim3(kThreads), lds, s, g, color, B,
                         chunks, coef, y, y_ld, rhs, rhs_ld, rhs_scale, rhs2, rhs2_ld, active,
                         part0, part1);
  });
  return chunks;
}
template int launch_gs_color<double, double>(const StencilGeom&, int, int, const double*, double*,
                                             int64_t, const double*, int64_t, const double*,
                                             const double*, int64_t, const int*, double*,
                                             double*, hipStream_t);
template int launch_gs_color<float, double>(const StencilGeom&, int, int, const double*, float*,
                                            int64_t, const double*, int64_t, const double*,
                                            const double*, int64_t, const int*, double*, double*,
                                            hipStream_t);
template int launch_gs_color<float, float>(const StencilGeom&, int, int, const double*, float*,
                                           int64_t, const float*, int64_t, const double*,
                                           const double*, int64_t, const int*, double*, double*,
                                           hipStream_t);

template <typename TY>
void launch_jacobi(const StencilGeom& g, int B, const double* coef, const TY* z, TY* y,
                   int64_t y_ld, double omega, const double* rhs, int64_t rhs_ld,
                   const double* rhs2, int64_t rhs2_ld, const int* active, double* part0,
                   double* part1, hipStream_t s) {
  if (g.csr)
    return csr_jacobi<TY>(g, B, coef, z, y, y_ld, omega, rhs, rhs_ld, rhs2, rhs2_ld, active,
                          part0, part1, s);
  const int chunks = stencil_chunks_all(g.N);
  const int qpb = pick_qpb(g, B, (int)sizeof(TY));
  dispatch(g.dim, qpb, [&](auto D, auto Q) {
    hipLaunchKernelGGL((k_jacobi<D.value, Q.value, TY>), grid_for(chunks, B, Q.value),
                       dim3(kThreads), Q.value * g.ct_size * (int)sizeof(TY), s, g, B, chunks,
                       coef, z, y, y_ld, omega, rhs, rhs_ld, rhs2, rhs2_ld, active, part0, part1);
  });
}
template void launch_jacobi<double>(const StencilGeom&, int, const double*, const double*,
                                    double*, int64_t, double, const double*, int64_t,
                                    const double*, int64_t, const int*, double*, double*,
                                    hipStream_t);
template void launch_jacobi<float>(const StencilGeom&, int, const double*, const float*, float*,
                                   int64_t, double, const double*, int64_t, const double*,
                                   int64_t, const int*, double*, double*, hipStream_t);

}  // namespace rb
