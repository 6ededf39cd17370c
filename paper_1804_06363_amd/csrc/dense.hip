// Reduced-basis contractions and reduced solves.
//
//  * projection   t_b = W^T r_b            (eq. 5; Alg. 2)         MFMA, split-K partials
//  * prolongation z_b = W e_b              (eq. 7; Alg. 2)         one node per thread
//  * reduced assembly + Cholesky  A_N(mu) = sum_q Theta_q A_{N,q} = L L^T  (eq. 12b, Sec. 2.1)
//  * reduced solve  e_b = L^-T L^-1 t_b    (eq. 6; Alg. 2)      
//  * deterministic finalisation of per-block partial sums and the CG scalars of Alg. 3
#include <hip/hip_runtime.h>

#include <algorithm>

#include "internal.h"
#include "kernels.h"

namespace rb {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef short shortx4 __attribute__((ext_vector_type(4)));

// ---- MFMA projection ---------------------------------------------------------------
// part[chunk][b][j] = sum_{k in chunk} W[j][k] r_b[k] for j < 16*JT.
// One wave owns a 16*QT (queries) x 16*JT (basis) tile of the product R W^T and walks
// its DOF range in steps of 16 with 16x16 MFMA tiles (queries = MFMA rows, basis
// vectors = MFMA columns).  Within a 16-DOF step lane l (row l%16, group g = l/16)
// supplies the four consecutive DOFs k0+4g..k0+4g+3, so each lane issues contiguous
// vector loads; for the K=4 instructions (FP32/FP64) sub-step s uses DOF k0+4g+s of
// both operands, for the K=16 BF16 instruction group g holds k0+4g..+3.  The
// summation order is fixed by the tiling, so results are deterministic.
// Vectors must be zero beyond N up to their stride (the library keeps them so).
template <typename TW>
struct ProjTraits;
template <>
struct ProjTraits<double> {
  using Acc = double;
  using Vec = doublex4;
};
template <>
struct ProjTraits<float> {
  using Acc = float;
  using Vec = floatx4;
};
template <>
struct ProjTraits<uint16_t> {
  using Acc = float;
  using Vec = floatx4;
};

// Row (within a 16-row tile) of accumulator register i held by lane group g: the FP32 /
// BF16 16x16 instructions give row 4g + i, the FP64 16x16x4 instruction row g + 4i.
template <typename TW>
__device__ __forceinline__ int acc_row(int g, int i) {
  return sizeof(TW) == 8 ? g + 4 * i : 4 * g + i;
}

// PADDED: R has a multiple of 16*QT rows and W round_up(n, 16) rows, zero beyond B and
// n, so the loads need no bounds checks (no branches between them).
// One step = 16 DOFs: lane (qi, kg) holds R[q_base + 16 t + qi][k0 + 4 kg .. +3] of every
// query tile t and W[16 u + qi][same DOFs] of every basis tile u.
// RT: type of the residual rows (double, or float for an FP32 copy with an FP32 / BF16
// basis: the products round the residual to FP32 first, so the result is the same)
template <typename TW, int QT, int JT, typename RT = double>
struct ProjFrag {
  RT a[QT][4];
  TW w[JT][4];
};

// row[t] / ok[t]: the residual row of this lane in query tile t and whether it is loaded
// (PADDED: always; rows are valid addresses either way).
template <typename TW, int QT, int JT, bool PADDED, typename RT>
__device__ __forceinline__ void proj_load(const RT* __restrict__ R, int64_t r_ld,
                                          const TW* __restrict__ W, int64_t w_ld, int n,
                                          const int (&row)[QT], const bool (&ok)[QT], int k0,
                                          ProjFrag<TW, QT, JT, RT>& f) {
  const int lane = threadIdx.x & 63;
  const int qi = lane & 15, kg = lane >> 4;
  const int kk = k0 + 4 * kg;
#pragma unroll
  for (int t = 0; t < QT; ++t) {
    if (PADDED || ok[t]) {
      if constexpr (sizeof(RT) == 8) {
        const double2* src = reinterpret_cast<const double2*>(R + (size_t)row[t] * r_ld + kk);
        const double2 v0 = src[0], v1 = src[1];
        f.a[t][0] = v0.x; f.a[t][1] = v0.y; f.a[t][2] = v1.x; f.a[t][3] = v1.y;
      } else {
        const float4 v = *reinterpret_cast<const float4*>(R + (size_t)row[t] * r_ld + kk);
        f.a[t][0] = v.x; f.a[t][1] = v.y; f.a[t][2] = v.z; f.a[t][3] = v.w;
      }
    } else {
      f.a[t][0] = f.a[t][1] = f.a[t][2] = f.a[t][3] = RT(0);
    }
  }
#pragma unroll
  for (int u = 0; u < JT; ++u) {
    const int j = 16 * u + qi;
    const TW* src = W + (size_t)j * w_ld + kk;
    if (PADDED || j < n) {
      if constexpr (sizeof(TW) == 8) {
        const double2 v0 = reinterpret_cast<const double2*>(src)[0];
        const double2 v1 = reinterpret_cast<const double2*>(src)[1];
        f.w[u][0] = v0.x; f.w[u][1] = v0.y; f.w[u][2] = v1.x; f.w[u][3] = v1.y;
      } else if constexpr (sizeof(TW) == 4) {
        const float4 v = *reinterpret_cast<const float4*>(src);
        f.w[u][0] = v.x; f.w[u][1] = v.y; f.w[u][2] = v.z; f.w[u][3] = v.w;
      } else {
        const uint2 v = *reinterpret_cast<const uint2*>(src);
        f.w[u][0] = (TW)(v.x & 0xffff); f.w[u][1] = (TW)(v.x >> 16);
        f.w[u][2] = (TW)(v.y & 0xffff); f.w[u][3] = (TW)(v.y >> 16);
      }
    } else {
      f.w[u][0] = f.w[u][1] = f.w[u][2] = f.w[u][3] = TW(0);
    }
  }
}

template <typename TW, int QT, int JT, typename RT>
__device__ __forceinline__ void proj_mma(const ProjFrag<TW, QT, JT, RT>& f,
                                         typename ProjTraits<TW>::Vec (&acc)[QT][JT]) {
  if constexpr (sizeof(TW) == 8) {  // FP64
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int t = 0; t < QT; ++t)
#pragma unroll
        for (int u = 0; u < JT; ++u)
          acc[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(f.a[t][s], f.w[u][s], acc[t][u], 0,
                                                           0, 0);
  } else if constexpr (sizeof(TW) == 4) {  // FP32 operands, FP32 accumulation
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int t = 0; t < QT; ++t)
#pragma unroll
        for (int u = 0; u < JT; ++u)
          acc[t][u] = __builtin_amdgcn_mfma_f32_16x16x4f32((float)f.a[t][s], f.w[u][s],
                                                           acc[t][u], 0, 0, 0);
  } else {  // BF16 operands, FP32 accumulation
    shortx4 w[JT];
#pragma unroll
    for (int u = 0; u < JT; ++u)
#pragma unroll
      for (int s = 0; s < 4; ++s) w[u][s] = (short)f.w[u][s];
#pragma unroll
    for (int t = 0; t < QT; ++t) {
      shortx4 av;
#pragma unroll
      for (int s = 0; s < 4; ++s) av[s] = (short)rbk::f32_to_bf16_rne((float)f.a[t][s]);
#pragma unroll
      for (int u = 0; u < JT; ++u)
        acc[t][u] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, w[u], acc[t][u], 0, 0, 0);
    }
  }
}

// WSPLIT = true: the block's 4 waves split the DOF range of one query tile and are
// reduced through LDS (small batches).  WSPLIT = false: the 4 waves own 4 query tiles
// over the same DOF range (large batches).
// qlist (batched path only, nullable): the active queries in increasing order, their
// count in qlist[B]; the wave tiles then run over that list (tiles past the count exit)
// and partial sums still go to the query's own row.
// WCH = true (wchunk plans): each wave covers all the group's queries (QT tiles) over a
// DOF range of its own; its partial sums are chunk 4 * blockIdx.x + wave.
template <typename TW, int QT, int JT, bool WSPLIT, bool PADDED, bool WCH = false,
          typename RT = double>
__global__ __launch_bounds__(256) void k_project(const RT* __restrict__ R, int64_t r_ld,
                                                 const TW* __restrict__ W, int64_t w_ld, int n,
                                                 int B, int kend, int steps,
                                                 const int* __restrict__ active,
                                                 const int* __restrict__ qlist,
                                                 typename ProjTraits<TW>::Acc* __restrict__ part) {
  using Acc = typename ProjTraits<TW>::Acc;
  using Vec = typename ProjTraits<TW>::Vec;
  constexpr int NJ = 16 * JT;
  constexpr int QW = 16 * QT;  // queries per wave tile
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int chunk = blockIdx.x;
  int q_base, k_begin, k_stop;
  if (WSPLIT) {
    q_base = blockIdx.y * QW;
    k_begin = (chunk * 4 + wave) * steps * 16;
  } else if (WCH) {
    q_base = 0;
    k_begin = (chunk * 4 + wave) * steps * 16;
  } else {
    q_base = (blockIdx.y * 4 + wave) * QW;
    k_begin = chunk * steps * 16;
  }
  k_stop = k_begin + steps * 16;
  if (k_stop > kend) k_stop = kend;
  // this lane's residual rows (no barriers in the batched path: a wave may leave alone)
  const int cnt = (!WSPLIT && qlist) ? qlist[B] : B;
  if (!WSPLIT && qlist && q_base >= cnt) return;
  int row[QT];
  bool ok[QT];
#pragma unroll
  for (int t = 0; t < QT; ++t) {
    const int c = q_base + 16 * t + (lane & 15);
    if (!WSPLIT && qlist) {
      row[t] = qlist[min(c, cnt - 1)];
      ok[t] = c < cnt;
    } else {
      row[t] = c;
      ok[t] = c < B && active[c];
    }
  }
  Vec acc[QT][JT];
#pragma unroll
  for (int t = 0; t < QT; ++t)
#pragma unroll
    for (int u = 0; u < JT; ++u) acc[t][u] = Vec{0, 0, 0, 0};
  // two fragments in fixed registers: step k+16 is loaded while step k multiplies (the
  // loop runs two steps per trip; a prefetch past the range reloads the last step)
  if (k_begin < k_stop) {
    const int klast = k_stop - 16;
    ProjFrag<TW, QT, JT, RT> f0, f1;
    proj_load<TW, QT, JT, PADDED>(R, r_ld, W, w_ld, n, row, ok, k_begin, f0);
    for (int k0 = k_begin; k0 < k_stop; k0 += 32) {
      proj_load<TW, QT, JT, PADDED>(R, r_ld, W, w_ld, n, row, ok, min(k0 + 16, klast), f1);
      proj_mma<TW, QT, JT>(f0, acc);
      if (k0 + 16 < k_stop) {
        proj_load<TW, QT, JT, PADDED>(R, r_ld, W, w_ld, n, row, ok, min(k0 + 32, klast), f0);
        proj_mma<TW, QT, JT>(f1, acc);
      }
    }
  }

  const int qi = lane & 15, kg = lane >> 4;
  if (!WSPLIT) {
    const int pchunk = WCH ? chunk * 4 + wave : chunk;
#pragma unroll
    for (int t = 0; t < QT; ++t)
#pragma unroll
      for (int u = 0; u < JT; ++u)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int c = q_base + 16 * t + acc_row<TW>(kg, i);
          const int j = 16 * u + qi;
          if (c < cnt) part[((size_t)pchunk * B + (qlist ? qlist[c] : c)) * NJ + j] = acc[t][u][i];
        }
  } else {
    __shared__ Acc sh[4][QW][NJ];
#pragma unroll
    for (int t = 0; t < QT; ++t)
#pragma unroll
      for (int u = 0; u < JT; ++u)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          sh[wave][16 * t + acc_row<TW>(kg, i)][16 * u + qi] = acc[t][u][i];
    __syncthreads();
    for (int e = threadIdx.x; e < QW * NJ; e += 256) {
      const int ql = e / NJ, j = e % NJ;
      const int q = q_base + ql;
      const Acc s = (sh[0][ql][j] + sh[1][ql][j]) + (sh[2][ql][j] + sh[3][ql][j]);
      if (q < B) part[((size_t)chunk * B + q) * NJ + j] = s;
    }
  }
}

ProjPlan plan_projection(int N, int B, int n, int target_blocks) {
  ProjPlan p;
  p.jt = (n + 15) / 16;
  if (p.jt < 1) p.jt = 1;
  p.kend = ((N + 15) / 16) * 16;
  const int nsteps = p.kend / 16;
  if (B <= 16) {
    p.wsplit = true;
    p.qt = 1;
    p.qgroups = (B + 15) / 16;
    // steps per wave so that chunks*qgroups ~ target
    // one block per CU is enough for a GEMV-like pass; fewer chunks keep the
    // finalising reduction short
    int chunks_wanted = std::min(target_blocks, 256) / p.qgroups;
    if (chunks_wanted < 1) chunks_wanted = 1;
    p.steps = (nsteps + 4 * chunks_wanted - 1) / (4 * chunks_wanted);
    if (p.steps < 1) p.steps = 1;
    p.chunks = (nsteps + 4 * p.steps - 1) / (4 * p.steps);
  } else {
    p.wsplit = false;
    p.qt = B <= 64 ? 1 : (B <= 128 ? 2 : 4);
    if (p.jt > 3 && p.qt > 2) p.qt = 2;  // register budget
    p.qgroups = (B + 64 * p.qt - 1) / (64 * p.qt);
    int chunks_wanted = target_blocks / p.qgroups;
    if (chunks_wanted < 1) chunks_wanted = 1;
    p.steps = (nsteps + chunks_wanted - 1) / chunks_wanted;
    if (p.steps < 1) p.steps = 1;
    p.chunks = (nsteps + p.steps - 1) / p.steps;
  }
  p.nj = 16 * p.jt;
  p.blocks = p.chunks;
  return p;
}

void plan_wave_chunks(ProjPlan& p, int B, int target_blocks, rb_prec prec) {
  // with at most 64 queries the four waves of a batched block hold four 16-query tiles
  // over the same DOFs and each loads the block's basis rows; with a large basis those
  // rows outweigh the residual rows, so one wave takes all queries instead (QT = 4; the
  // FP64 basis would not fit the registers)
  if (p.wsplit || !p.padded || B <= 16 || B > 64 || p.jt < 4 || prec == RB_PREC_FP64) return;
  const int nsteps = p.kend / 16;
  // two waves per block-target unit: the default target (four blocks per CU) then gives
  // two of these register-heavy waves per SIMD
  const int waves = std::max(4, 2 * target_blocks);
  p.wchunk = true;
  p.qt = 4;
  p.qgroups = 1;
  p.steps = std::max(1, (nsteps + waves - 1) / waves);
  const int used = (nsteps + p.steps - 1) / p.steps;  // waves with DOFs
  p.blocks = (used + 3) / 4;
  p.chunks = 4 * p.blocks;
}

template <typename TW, int QT, int JT, typename RT>
static void launch_proj_t(const ProjPlan& pl, const RT* R, int64_t r_ld, const TW* W,
                          int64_t w_ld, int n, int B, const int* active, const int* qlist,
                          void* part, hipStream_t s) {
  using Acc = typename ProjTraits<TW>::Acc;
  const dim3 grid(pl.blocks, pl.qgroups);
  if constexpr (QT == 4 && sizeof(TW) < 8) {
    if (pl.wchunk) {
      hipLaunchKernelGGL((k_project<TW, QT, JT, false, true, true, RT>), grid, dim3(256), 0, s,
                         R, r_ld, W, w_ld, n, B, pl.kend, pl.steps, active, qlist, (Acc*)part);
      return;
    }
  }
  RB_REQUIRE(!pl.wchunk, RB_EUNSUPPORTED, "wave-chunk projection plan for an FP64 basis");
  if (pl.wsplit)
    hipLaunchKernelGGL((k_project<TW, QT, JT, true, false, false, RT>), grid, dim3(256), 0, s, R,
                       r_ld, W, w_ld, n, B, pl.kend, pl.steps, active, nullptr, (Acc*)part);
  else if (pl.padded)
    hipLaunchKernelGGL((k_project<TW, QT, JT, false, true, false, RT>), grid, dim3(256), 0, s, R,
                       r_ld, W, w_ld, n, B, pl.kend, pl.steps, active, qlist, (Acc*)part);
  else
    hipLaunchKernelGGL((k_project<TW, QT, JT, false, false, false, RT>), grid, dim3(256), 0, s, R,
                       r_ld, W, w_ld, n, B, pl.kend, pl.steps, active, qlist, (Acc*)part);
}

template <typename TW, int QT, typename RT>
static void launch_proj_q(const ProjPlan& pl, const RT* R, int64_t r_ld, const TW* W,
                          int64_t w_ld, int n, int B, const int* active, const int* ql,
                          void* part, hipStream_t s) {
  switch (pl.jt) {
    case 1: launch_proj_t<TW, QT, 1>(pl, R, r_ld, W, w_ld, n, B, active, ql, part, s); break;
    case 2: launch_proj_t<TW, QT, 2>(pl, R, r_ld, W, w_ld, n, B, active, ql, part, s); break;
    case 3: launch_proj_t<TW, QT, 3>(pl, R, r_ld, W, w_ld, n, B, active, ql, part, s); break;
    case 4: launch_proj_t<TW, QT, 4>(pl, R, r_ld, W, w_ld, n, B, active, ql, part, s); break;
    default: launch_proj_t<TW, QT, 5>(pl, R, r_ld, W, w_ld, n, B, active, ql, part, s); break;
  }
}

template <typename TW, typename RT>
static void launch_proj_w(const ProjPlan& pl, const RT* R, int64_t r_ld, const void* W,
                          int64_t w_ld, int n, int B, const int* active, const int* ql,
                          void* part, hipStream_t s) {
  const TW* w = (const TW*)W;
  switch (pl.qt) {
    case 1: launch_proj_q<TW, 1>(pl, R, r_ld, w, w_ld, n, B, active, ql, part, s); break;
    case 2: launch_proj_q<TW, 2>(pl, R, r_ld, w, w_ld, n, B, active, ql, part, s); break;
    default: launch_proj_q<TW, 4>(pl, R, r_ld, w, w_ld, n, B, active, ql, part, s); break;
  }
}

void launch_projection(const ProjPlan& pl, rb_prec prec, const double* R, int64_t r_ld,
                       const void* W, int64_t w_ld, int n, int B, const int* active, void* part,
                       hipStream_t s, const int* qlist, const float* R32) {
  if (prec == RB_PREC_FP64)
    launch_proj_w<double>(pl, R, r_ld, W, w_ld, n, B, active, qlist, part, s);
  else if (prec == RB_PREC_FP32 && R32)
    launch_proj_w<float>(pl, R32, r_ld, W, w_ld, n, B, active, qlist, part, s);
  else if (prec == RB_PREC_FP32)
    launch_proj_w<float>(pl, R, r_ld, W, w_ld, n, B, active, qlist, part, s);
  else if (R32)
    launch_proj_w<uint16_t>(pl, R32, r_ld, W, w_ld, n, B, active, qlist, part, s);
  else
    launch_proj_w<uint16_t>(pl, R, r_ld, W, w_ld, n, B, active, qlist, part, s);
}

// ---- prolongation -----------------------------------------------------------------
// out_b[pos] (=|+=) sum_{j<n} W[j][pos] e_b[j] for pos in [lo, hi); QG queries per
// block (blockIdx.x = query group, blockIdx.y = node chunk).  e rows are zero beyond a
// query's own basis size.
template <typename TW, typename TA, typename TO, int QG, bool ADD>
__global__ __launch_bounds__(256) void k_prolong(const TW* __restrict__ W, int64_t w_ld, int n,
                                                 const TA* __restrict__ e, int e_ld, int B,
                                                 const int* __restrict__ active,
                                                 TO* __restrict__ out, int64_t o_ld, int lo,
                                                 int hi) {
  const int q0 = blockIdx.x * QG;
  const int pos = lo + blockIdx.y * 256 + threadIdx.x;
  if (pos >= hi) return;
  TA acc[QG];
#pragma unroll
  for (int q = 0; q < QG; ++q) acc[q] = TA(0);
  for (int j = 0; j < n; ++j) {
    TA w;
    if constexpr (sizeof(TW) == 2)
      w = (TA)rbk::bf16_to_f32(W[(size_t)j * w_ld + pos]);
    else
      w = (TA)W[(size_t)j * w_ld + pos];
#pragma unroll
    for (int q = 0; q < QG; ++q) acc[q] += w * e[(size_t)(q0 + q) * e_ld + j];
  }
#pragma unroll
  for (int q = 0; q < QG; ++q) {
    const int b = q0 + q;
    if (b < B && active[b]) {
      TO* o = out + (size_t)b * o_ld + pos;
      if (ADD)
        *o += (TO)acc[q];
      else
        *o = (TO)acc[q];
    }
  }
}

// Batched prolongation on MFMA (FP32 / BF16 bases, B >= 16): the product
// Z[q][pos] = sum_j e_q[j] W[j][pos] as 16x16 MFMA tiles with queries as rows and
// nodes as columns, K = basis index in steps of 4 (v_mfma_f32_16x16x4f32; BF16 basis
// entries widen exactly to FP32).  A block is 4 waves x 16 queries over a run of
// 16*TP consecutive nodes: every wave writes 64*TP contiguous bytes per query row
// (DRAM-friendly) and the block's waves share the W tile through L1.  Lane l supplies
// e[q0 + l%16][j0 + l/16] and, for MFMA block p = 4k + u, W[j0 + l/16][pos0 + 64k +
// 4(l%16) + u], and receives rows 4(l/16)+i (queries) of that column (node): its W
// loads and its stores are 4 consecutive nodes wide (127^3, B = 256, FP32: 454 us per
// launch against 512 us with one node per access).  Blocks are remapped so that the
// query groups of one node run sit on one XCD (their W tile is fetched once).
template <typename TW, typename TO, int TP, bool ADD>
// qlist (nullable): the active queries in increasing order, their count in qlist[B]; the
// query groups then run over that list (groups past the count exit).
__global__ __launch_bounds__(256) void k_prolong_mfma(const TW* __restrict__ W, int64_t w_ld, int n,
                                                      const float* __restrict__ e, int e_ld, int B,
                                                      const int* __restrict__ active,
                                                      const int* __restrict__ qlist,
                                                      TO* __restrict__ out, int64_t o_ld, int lo,
                                                      int hi, int qgroups) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // XCD-aware remap of the 1D grid: consecutive remapped ids share the node run
  const int total = gridDim.x;
  const int qd = total / 8, rd = total % 8;
  const int xcd = blockIdx.x % 8, slot = blockIdx.x / 8;
  const int id = xcd < rd ? xcd * (qd + 1) + slot : rd * (qd + 1) + (xcd - rd) * qd + slot;
  const int run = id / qgroups, qg = id % qgroups;
  const int cnt = qlist ? qlist[B] : B;
  if (qg * 64 >= cnt) return;  // no barriers in this kernel
  // runs start at lo rounded down to a multiple of 4 (nodes below lo are not stored)
  const int pos0 = (lo & ~3) + run * 16 * TP;
  const int q0 = (qg * 4 + wave) * 16;
  const int r = lane & 15, g = lane >> 4;
  // e row of this lane: its query (through the list; past the count any valid row, whose
  // results are not stored)
  const int erow = qlist ? qlist[min(q0 + r, cnt - 1)] : q0 + r;
  floatx4 acc[TP];
#pragma unroll
  for (int p = 0; p < TP; ++p) acc[p] = floatx4{0.f, 0.f, 0.f, 0.f};
  // Column r of MFMA block p = 4k + u is node pos0 + 64k + 4r + u, so a lane loads the
  // W entries of four blocks, and stores their results, as four consecutive nodes.
  // Loads are unconditional: the caller pads e to round_up(B, 64) zero rows and at
  // least round_up(n, 4) columns, and W to round_up(n, 4) + 1 rows (zero beyond n),
  // so every address is inside its buffer; nodes outside [lo, hi) are not stored.
  for (int j0 = 0; j0 < n; j0 += 4) {
    const int j = j0 + g;
    const float ev = e[(size_t)erow * e_ld + j];
    const TW* wr = W + (size_t)j * w_ld + pos0 + 4 * r;
#pragma unroll
    for (int k = 0; k < TP / 4; ++k) {
      float wv[4];
      if constexpr (sizeof(TW) == 2) {
        const uint2 v = *reinterpret_cast<const uint2*>(wr + 64 * k);
        wv[0] = rbk::bf16_to_f32((uint16_t)(v.x & 0xffff));
        wv[1] = rbk::bf16_to_f32((uint16_t)(v.x >> 16));
        wv[2] = rbk::bf16_to_f32((uint16_t)(v.y & 0xffff));
        wv[3] = rbk::bf16_to_f32((uint16_t)(v.y >> 16));
      } else {
        const float4 v = *reinterpret_cast<const float4*>(wr + 64 * k);
        wv[0] = v.x; wv[1] = v.y; wv[2] = v.z; wv[3] = v.w;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        acc[4 * k + u] = __builtin_amdgcn_mfma_f32_16x16x4f32(ev, wv[u], acc[4 * k + u], 0, 0, 0);
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int c = q0 + 4 * g + i;
    if (c >= cnt) continue;
    const int q = qlist ? qlist[c] : c;
    if (!qlist && !active[q]) continue;
    TO* o = out + (size_t)q * o_ld;
#pragma unroll
    for (int k = 0; k < TP / 4; ++k) {
      const int p0 = pos0 + 64 * k + 4 * r;
      if (!ADD && p0 >= lo && p0 + 3 < hi) {
        if constexpr (sizeof(TO) == 4) {
          *reinterpret_cast<float4*>(o + p0) =
              float4{acc[4 * k][i], acc[4 * k + 1][i], acc[4 * k + 2][i], acc[4 * k + 3][i]};
        } else {
          reinterpret_cast<double2*>(o + p0)[0] =
              double2{(double)acc[4 * k][i], (double)acc[4 * k + 1][i]};
          reinterpret_cast<double2*>(o + p0)[1] =
              double2{(double)acc[4 * k + 2][i], (double)acc[4 * k + 3][i]};
        }
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int pos = p0 + u;
          if (pos >= lo && pos < hi) {
            if (ADD)
              o[pos] += (TO)acc[4 * k + u][i];
            else
              o[pos] = (TO)acc[4 * k + u][i];
          }
        }
      }
    }
  }
}

// Batched prolongation on the vector units (FP32 / BF16 basis, FP32 arithmetic, out
// overwritten): one node per thread.  The thread holds its node's NB = round_up(n, 8) basis
// entries in registers and forms out_q[pos] = sum_{j<n} W[j][pos] e_q[j], j in increasing
// order, for the queries of its block's chunk, two at a time.  The e rows are the same for
// every lane (block-uniform addresses), so they come through the scalar cache into scalar
// registers and each product is one FMA with a scalar operand; each store writes 256
// consecutive entries of one query's row.  A run of 256 nodes is read once per query chunk,
// and the chunks of a run are consecutive block ids on one XCD, so the later ones find its
// W rows in L2.  Against the MFMA kernel this issues all of a node's W loads at once
// instead of one four-row step after another.
constexpr int kVecQChunk = 64;  // queries per block
template <typename TW, typename TO, int NB>
__global__ __launch_bounds__(256) void k_prolong_vec(const TW* __restrict__ W, int64_t w_ld, int n,
                                                     const float* __restrict__ e, int e_ld,
                                                     int B, const int* __restrict__ active,
                                                     const int* __restrict__ qlist,
                                                     TO* __restrict__ out, int64_t o_ld, int lo,
                                                     int hi, int qchunks) {
  const int total = gridDim.x;
  const int qd = total / 8, rd = total % 8;
  const int xcd = blockIdx.x % 8, slot = blockIdx.x / 8;
  const int id = xcd < rd ? xcd * (qd + 1) + slot : rd * (qd + 1) + (xcd - rd) * qd + slot;
  const int run = id / qchunks, qc = id % qchunks;
  const int cnt = qlist ? qlist[B] : B;
  const int c0 = qc * kVecQChunk;
  if (c0 >= cnt) return;
  const int c1 = min(c0 + kVecQChunk, cnt);
  const int pos = lo + run * 256 + (int)threadIdx.x;
  const bool ok = pos < hi;
  const int pc = ok ? pos : lo;  // a valid address for the loads of lanes past hi
  // rows below NB - 8 exist (n > NB - 8); the last eight load row min(j, n - 1) and keep
  // zero past n, so every load is unconditional and in bounds
  float w[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const int jr = (j < NB - 8 || j < n) ? j : n - 1;
    float v;
    if constexpr (sizeof(TW) == 2)
      v = rbk::bf16_to_f32(W[(size_t)jr * w_ld + pc]);
    else
      v = (float)W[(size_t)jr * w_ld + pc];
    w[j] = (j < NB - 8 || j < n) ? v : 0.f;
  }
  for (int c = c0; c < c1; c += 2) {
    const bool two = c + 1 < c1;
    const int qa = qlist ? qlist[c] : c;
    const int qb = two ? (qlist ? qlist[c + 1] : c + 1) : qa;
    const float* ea = e + (size_t)qa * e_ld;
    const float* eb = e + (size_t)qb * e_ld;
    float a = 0.f, b = 0.f;
#pragma unroll
    for (int j0 = 0; j0 < NB; j0 += 8) {
      // eight entries of each e row at a time: the compiler barrier keeps the scalar loads
      // of later entries from being hoisted here, which would exhaust the scalar registers
      asm volatile("" ::: "memory");
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int j = j0 + k;
        if (j0 + 8 < NB || j < n) {  // only the last group of eight can pass n
          a = fmaf(w[j], ea[j], a);
          b = fmaf(w[j], eb[j], b);
        }
      }
    }
    if (ok && (qlist || active[qa])) out[(size_t)qa * o_ld + pos] = (TO)a;
    if (two && ok && (qlist || active[qb])) out[(size_t)qb * o_ld + pos] = (TO)b;
  }
}

template <typename TW, typename TO>
static void launch_prolong_vec(const TW* W, int64_t w_ld, int n, const float* e, int e_ld, int B,
                               const int* active, const int* qlist, TO* out, int64_t o_ld, int lo,
                               int hi, hipStream_t s) {
  const int runs = (hi - lo + 255) / 256;
  const int qchunks = (B + kVecQChunk - 1) / kVecQChunk;
  const dim3 grid((unsigned)(runs * qchunks));
  auto go = [&](auto NBc) {
    hipLaunchKernelGGL((k_prolong_vec<TW, TO, NBc.value>), grid, dim3(256), 0, s, W, w_ld, n, e,
                       e_ld, B, active, qlist, out, o_ld, lo, hi, qchunks);
  };
  switch ((n + 7) / 8) {
    case 1: go(std::integral_constant<int, 8>{}); break;
    case 2: go(std::integral_constant<int, 16>{}); break;
    case 3: go(std::integral_constant<int, 24>{}); break;
    case 4: go(std::integral_constant<int, 32>{}); break;
    case 5: go(std::integral_constant<int, 40>{}); break;
    case 6: go(std::integral_constant<int, 48>{}); break;
    case 7: go(std::integral_constant<int, 56>{}); break;
    case 8: go(std::integral_constant<int, 64>{}); break;
    case 9: go(std::integral_constant<int, 72>{}); break;
    default:
      RB_REQUIRE(n <= 80, RB_EUNSUPPORTED, "vector prolongation: basis size above 80");
      go(std::integral_constant<int, 80>{});
      break;
  }
}

template <typename TW, typename TO, bool ADD>
static void launch_prolong_mfma(const TW* W, int64_t w_ld, int n, const float* e, int e_ld, int B,
                                const int* active, const int* qlist, TO* out, int64_t o_ld,
                                int lo, int hi, hipStream_t s) {
  constexpr int TP = 16;
  static_assert(TP % 4 == 0, "four MFMA blocks per vector access");
  const int runs = (hi - (lo & ~3) + 16 * TP - 1) / (16 * TP);
  const int qgroups = (B + 63) / 64;
  hipLaunchKernelGGL((k_prolong_mfma<TW, TO, TP, ADD>), dim3(runs * qgroups), dim3(256), 0, s, W,
                     w_ld, n, e, e_ld, B, active, qlist, out, o_ld, lo, hi, qgroups);
}

template <typename TW, typename TA, typename TO, bool ADD>
static void launch_prolong_t(const TW* W, int64_t w_ld, int n, const TA* e, int e_ld, int B,
                             const int* active, TO* out, int64_t o_ld, int lo, int hi,
                             hipStream_t s) {
  constexpr int QG = 8;
  const dim3 grid((B + QG - 1) / QG, (hi - lo + 255) / 256);
  hipLaunchKernelGGL((k_prolong<TW, TA, TO, QG, ADD>), grid, dim3(256), 0, s, W, w_ld, n, e, e_ld,
                     B, active, out, o_ld, lo, hi);
}

void launch_prolong(rb_prec prec, const void* W, int64_t w_ld, int n, const double* e64,
                    const float* e32, int e_ld, int B, const int* active, void* out,
                    bool out_is_double, int64_t o_ld, int lo, int hi, bool add, hipStream_t s,
                    const int* qlist) {
  if (hi <= lo || n == 0) return;
  if (prec == RB_PREC_FP64) {
    RB_REQUIRE(out_is_double, RB_EINVAL, "FP64 prolongation needs a double output");
    if (add)
      launch_prolong_t<double, double, double, true>((const double*)W, w_ld, n, e64, e_ld, B,
                                                     active, (double*)out, o_ld, lo, hi, s);
    else
      launch_prolong_t<double, double, double, false>((const double*)W, w_ld, n, e64, e_ld, B,
                                                      active, (double*)out, o_ld, lo, hi, s);
    return;
  }
  if (B >= 16 && !add && stencil_tiles().kind_pro == 2) {
    if (prec == RB_PREC_FP32) {
      if (out_is_double)
        launch_prolong_vec<float, double>((const float*)W, w_ld, n, e32, e_ld, B, active, qlist,
                                          (double*)out, o_ld, lo, hi, s);
      else
        launch_prolong_vec<float, float>((const float*)W, w_ld, n, e32, e_ld, B, active, qlist,
                                         (float*)out, o_ld, lo, hi, s);
    } else {
      if (out_is_double)
        launch_prolong_vec<uint16_t, double>((const uint16_t*)W, w_ld, n, e32, e_ld, B, active,
                                             qlist, (double*)out, o_ld, lo, hi, s);
      else
        launch_prolong_vec<uint16_t, float>((const uint16_t*)W, w_ld, n, e32, e_ld, B, active,
                                            qlist, (float*)out, o_ld, lo, hi, s);
    }
    return;
  }
  if (B >= 16) {
#define PM(TW)                                                                                    \
  if (out_is_double) {                                                                            \
    if (add)                                                                                      \
      launch_prolong_mfma<TW, double, true>((const TW*)W, w_ld, n, e32, e_ld, B, active, qlist,   \
                                            (double*)out, o_ld, lo, hi, s);                       \
    else                                                                                          \
      launch_prolong_mfma<TW, double, false>((const TW*)W, w_ld, n, e32, e_ld, B, active,         \
                                             qlist, (double*)out, o_ld, lo, hi, s);               \
  } else {                                                                                        \
    if (add)                                                                                      \
      launch_prolong_mfma<TW, float, true>((const TW*)W, w_ld, n, e32, e_ld, B, active, qlist,    \
                                           (float*)out, o_ld, lo, hi, s);                         \
    else                                                                                          \
      launch_prolong_mfma<TW, float, false>((const TW*)W, w_ld, n, e32, e_ld, B, active, qlist,   \
                                            (float*)out, o_ld, lo, hi, s);                        \
  }
    if (prec == RB_PREC_FP32) {
      PM(float)
    } else {
      PM(uint16_t)
    }
#undef PM
    return;
  }
#define PR(TW)                                                                                   \
  if (out_is_double) {                                                                           \
    if (add)                                                                                     \
      launch_prolong_t<TW, float, double, true>((const TW*)W, w_ld, n, e32, e_ld, B, active,     \
                                                (double*)out, o_ld, lo, hi, s);                  \
    else                                                                                         \
      launch_prolong_t<TW, float, double, false>((const TW*)W, w_ld, n, e32, e_ld, B, active,    \
                                                 (double*)out, o_ld, lo, hi, s);                 \
  } else {                                                                                       \
    if (add)                                                                                     \
      launch_prolong_t<TW, float, float, true>((const TW*)W, w_ld, n, e32, e_ld, B, active,      \
                                               (float*)out, o_ld, lo, hi, s);                    \
    else                                                                                         \
      launch_prolong_t<TW, float, float, false>((const TW*)W, w_ld, n, e32, e_ld, B, active,     \
                                                (float*)out, o_ld, lo, hi, s);                   \
  }
  if (prec == RB_PREC_FP32) {
    PR(float)
  } else {
    PR(uint16_t)
  }
#undef PR
}

// ---- reduced assembly + Cholesky (one wavefront per query) --------------------------
// Right-looking unpivoted Cholesky of the leading nb x nb block of A (LDS, lower part
// overwritten by L) by one wavefront.  Returns true on a non-positive (or NaN) pivot.
template <int NMAX>
__device__ bool chol_lds(double (*A)[NMAX + 1], int nb, int lane, int* bad) {
  if (lane == 0) *bad = 0;
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    const double d = A[j][j];
    if (!(d > 0.0)) {
      if (lane == 0) *bad = 1;
      break;
    }
    const double ljj = sqrt(d);
    __syncthreads();
    if (lane == 0) A[j][j] = ljj;
    for (int i = j + 1 + lane; i < nb; i += 64) A[i][j] /= ljj;
    __syncthreads();
    // trailing update of the lower triangle: A[i][k] -= L[i][j] L[k][j], j < k <= i
    const int m = nb - j - 1;
    for (int e = lane; e < m * m; e += 64) {
      const int i = j + 1 + e / m, k = j + 1 + e % m;
      if (k <= i) A[i][k] -= A[i][j] * A[k][j];
    }
    __syncthreads();
  }
  __syncthreads();
  return *bad != 0;
}

// A = sum_q theta_bq A_{N,q} restricted to the leading n_b x n_b block.  L is written
// row-major [b][n][n] with zeros above the diagonal and outside n_b.  status[b] =
// RB_ENOTSPD on a non-positive (or NaN) pivot.
template <int NMAX>
__global__ __launch_bounds__(64) void k_cholesky(const double* __restrict__ AN, int n, int Q,
                                                 const double* __restrict__ theta,
                                                 const int* __restrict__ n_use,
                                                 double* __restrict__ L, int* __restrict__ status) {
  __shared__ double A[NMAX][NMAX + 1];
  __shared__ int bad;
  const int b = blockIdx.x;
  const int nb = n_use ? n_use[b] : n;
  const double* th = theta + (size_t)b * Q;
  const int lane = threadIdx.x;
  for (int e = lane; e < nb * nb; e += 64) {
    const int i = e / nb, j = e % nb;
    double s = 0.0;
    for (int q = 0; q < Q; ++q) s += th[q] * AN[((size_t)q * n + i) * n + j];
    A[i][j] = s;
  }
  __syncthreads();
  const bool fail = chol_lds<NMAX>(A, nb, lane, &bad);
  double* Lb = L + (size_t)b * n * n;
  for (int e = lane; e < n * n; e += 64) {
    const int i = e / n, j = e % n;
    Lb[e] = (i < nb && j <= i && !fail) ? A[i][j] : 0.0;
  }
  if (lane == 0) status[b] = fail ? (int)RB_ENOTSPD : (int)RB_OK;
}

// Greedy sweep of Alg. 4 (reduced solve and indicator): for candidate m, a(mu_m) = A_N(mu_m)^-1 f_N(mu_m)
// (assembly by eq. 12b, Cholesky, two triangular solves) and the L1 indicator
// sum_n |a_n|.  a rows have stride a_ld; status[m] = RB_ENOTSPD on failure (l1 = NaN).
template <int NMAX>
__global__ __launch_bounds__(64) void k_sweep_coeffs(const double* __restrict__ AN,
                                                     const double* __restrict__ fN, int n, int Q,
                                                     int R, const double* __restrict__ theta,
                                                     const double* __restrict__ phi,
                                                     double* __restrict__ a, int a_ld,
                                                     double* __restrict__ l1,
                                                     int* __restrict__ status) {
  __shared__ double A[NMAX][NMAX + 1];
  __shared__ double u[NMAX];
  __shared__ int bad;
  const int m = blockIdx.x;
  const int lane = threadIdx.x;
  const double* th = theta + (size_t)m * Q;
  for (int e = lane; e < n * n; e += 64) {
    const int i = e / n, j = e % n;
    double s = 0.0;
    for (int q = 0; q < Q; ++q) s += th[q] * AN[((size_t)q * n + i) * n + j];
    A[i][j] = s;
  }
  for (int j = lane; j < n; j += 64) {
    double s = 0.0;
    for (int r = 0; r < R; ++r) s += (phi ? phi[(size_t)m * R + r] : 1.0) * fN[(size_t)r * n + j];
    u[j] = s;
  }
  __syncthreads();
  const bool fail = chol_lds<NMAX>(A, n, lane, &bad);
  if (!fail) {
    for (int j = 0; j < n; ++j) {  // L v = f_N
      const double vj = u[j] / A[j][j];
      __syncthreads();
      if (lane == 0) u[j] = vj;
      for (int i = j + 1 + lane; i < n; i += 64) u[i] -= A[i][j] * vj;
      __syncthreads();
    }
    for (int j = n - 1; j >= 0; --j) {  // L^T a = v
      const double aj = u[j] / A[j][j];
      __syncthreads();
      if (lane == 0) u[j] = aj;
      for (int i = lane; i < j; i += 64) u[i] -= A[j][i] * aj;
      __syncthreads();
    }
  }
  double s1 = 0.0;
  for (int j = lane; j < a_ld; j += 64) {
    const double v = (j < n && !fail) ? u[j] : 0.0;
    a[(size_t)m * a_ld + j] = v;
    s1 += fabs(v);
  }
  s1 = rbk::wave_sum(s1);
  if (lane == 0) {
    l1[m] = fail ? __builtin_nan("") : s1;
    status[m] = fail ? (int)RB_ENOTSPD : (int)RB_OK;
  }
}

void launch_sweep_coeffs(const double* AN, const double* fN, int n, int Q, int R, int M,
                         const double* theta, const double* phi, double* a, int a_ld, double* l1,
                         int* status, hipStream_t s) {
  RB_REQUIRE(n >= 1 && n <= 80, RB_EUNSUPPORTED, "reduced basis size must be 1..80");
  if (n <= 32)
    hipLaunchKernelGGL(k_sweep_coeffs<32>, dim3(M), dim3(64), 0, s, AN, fN, n, Q, R, theta, phi, a,
                       a_ld, l1, status);
  else
    hipLaunchKernelGGL(k_sweep_coeffs<80>, dim3(M), dim3(64), 0, s, AN, fN, n, Q, R, theta, phi, a,
                       a_ld, l1, status);
}

// Masked argmax over M values (the next sample of Alg. 4): largest value among the entries with
// excluded[m] == 0; ties go to the lowest index.  out_val/out_idx; out_idx = -1 if every
// entry is excluded; nan_flag = 1 if a non-excluded entry is NaN.
__global__ __launch_bounds__(256) void k_argmax(const double* __restrict__ v,
                                                const int* __restrict__ excluded, int M,
                                                double* __restrict__ out_val,
                                                int* __restrict__ out_idx,
                                                int* __restrict__ nan_flag) {
  __shared__ double sv[256];
  __shared__ int si[256];
  __shared__ int snan;
  if (threadIdx.x == 0) snan = 0;
  __syncthreads();
  double best = -__builtin_inf();
  int bi = -1;
  for (int m = threadIdx.x; m < M; m += 256) {
    if (excluded[m]) continue;
    const double x = v[m];
    if (!(x == x)) {
      snan = 1;
      continue;
    }
    if (bi < 0 || x > best) {  // strictly greater keeps the lowest index of a tie
      best = x;
      bi = m;
    }
  }
  sv[threadIdx.x] = best;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int off = 128; off >= 1; off >>= 1) {
    if (threadIdx.x < off) {
      const double ov = sv[threadIdx.x + off];
      const int oi = si[threadIdx.x + off];
      const int ci = si[threadIdx.x];
      if (oi >= 0 && (ci < 0 || ov > sv[threadIdx.x] || (ov == sv[threadIdx.x] && oi < ci))) {
        sv[threadIdx.x] = ov;
        si[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *out_val = sv[0];
    *out_idx = si[0];
    *nan_flag = snan;
  }
}
void launch_argmax(const double* v, const int* excluded, int M, double* out_val, int* out_idx,
                   int* nan_flag, hipStream_t s) {
  hipLaunchKernelGGL(k_argmax, dim3(1), dim3(256), 0, s, v, excluded, M, out_val, out_idx,
                     nan_flag);
}

// partial sums of a_b . c_b over chunks of 256*per_thread entries: part[b][chunk]
__global__ __launch_bounds__(256) void k_dot(const double* __restrict__ a,
                                             const double* __restrict__ c, int64_t ld, int N,
                                             double* __restrict__ part, int per_thread) {
  __shared__ double sh[4];
  const int b = blockIdx.y;
  double acc = 0.0;
  const int base = blockIdx.x * 256 * per_thread;
  for (int t = 0; t < per_thread; ++t) {
    const int i = base + t * 256 + threadIdx.x;
    if (i >= N) break;
    acc += a[(size_t)b * ld + i] * c[(size_t)b * ld + i];
  }
  const double s = rbk::block_sum_256(acc, sh);
  if (threadIdx.x == 0) part[(size_t)b * gridDim.x + blockIdx.x] = s;
}
int launch_dot(const double* a, const double* c, int64_t ld, int N, int B, double* part,
               int per_thread, hipStream_t s) {
  const int chunks = (N + 256 * per_thread - 1) / (256 * per_thread);
  hipLaunchKernelGGL(k_dot, dim3(chunks, B), dim3(256), 0, s, a, c, ld, N, part, per_thread);
  return chunks;
}

// dst[i] = alpha * src[i]
__global__ void k_scale(double* __restrict__ dst, const double* __restrict__ src, int64_t n,
                        double alpha) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = alpha * src[i];
}
void launch_scale(double* dst, const double* src, int64_t n, double alpha, hipStream_t s) {
  int bx = (int)((n + 255) / 256);
  if (bx > 8192) bx = 8192;
  if (bx < 1) bx = 1;
  hipLaunchKernelGGL(k_scale, dim3(bx), dim3(256), 0, s, dst, src, n, alpha);
}

void launch_cholesky(const double* AN, int n, int Q, int B, const double* theta, const int* n_use,
                     double* L, int* status, hipStream_t s) {
  RB_REQUIRE(n <= 80, RB_EUNSUPPORTED, "reduced basis larger than 80");
  if (n <= 32)
    hipLaunchKernelGGL(k_cholesky<32>, dim3(B), dim3(64), 0, s, AN, n, Q, theta, n_use, L, status);
  else
    hipLaunchKernelGGL(k_cholesky<80>, dim3(B), dim3(64), 0, s, AN, n, Q, theta, n_use, L, status);
}

// ---- finalise projection partials + reduced solve --------------------------------------
// t_b[j] = sum over chunks (fixed order, FP64), then e_b = L_b^-T L_b^-1 t_b.
// One block of 256 threads per query: the 4 waves sum interleaved chunks, then wave 0
// solves.  e64 / e32 rows have stride e_ld and are zero for j >= n_b.
template <typename Acc>
__global__ __launch_bounds__(256) void k_reduce_solve(const Acc* __restrict__ part, int chunks,
                                                      int B, int nj, int n,
                                                      const int* __restrict__ n_use,
                                                      const double* __restrict__ L,
                                                      const int* __restrict__ active,
                                                      double* __restrict__ t_out,
                                                      double* __restrict__ e64,
                                                      float* __restrict__ e32, int e_ld,
                                                      int solve) {
  __shared__ double sh[4][128];
  __shared__ double u[128];
  const int b = blockIdx.x;
  if (active && !active[b]) return;
  const int nb = n_use ? n_use[b] : n;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int j = lane; j < nj; j += 64) {
    double s = 0.0;
#pragma unroll 8
    for (int c = wave; c < chunks; c += 4) s += (double)part[((size_t)c * B + b) * nj + j];
    sh[wave][j] = s;
  }
  __syncthreads();
  // wave 0 does the solve; the other waves only take part in the barriers
  const bool w0 = wave == 0;
  if (w0)
    for (int j = lane; j < nj; j += 64) {
      const double t = (sh[0][j] + sh[1][j]) + (sh[2][j] + sh[3][j]);
      u[j] = j < nb ? t : 0.0;
      if (t_out && j < n) t_out[(size_t)b * n + j] = t;
    }
  __syncthreads();
  if (solve) {
    const double* Lb = L + (size_t)b * n * n;
    // forward: L v = t (column oriented)
    for (int j = 0; j < nb; ++j) {
      const double vj = u[j] / Lb[(size_t)j * n + j];
      __syncthreads();
      if (w0) {
        if (lane == 0) u[j] = vj;
        for (int i = j + 1 + lane; i < nb; i += 64) u[i] -= Lb[(size_t)i * n + j] * vj;
      }
      __syncthreads();
    }
    // backward: L^T e = v
    for (int j = nb - 1; j >= 0; --j) {
      const double ej = u[j] / Lb[(size_t)j * n + j];
      __syncthreads();
      if (w0) {
        if (lane == 0) u[j] = ej;
        for (int i = lane; i < j; i += 64) u[i] -= Lb[(size_t)j * n + i] * ej;
      }
      __syncthreads();
    }
  }
  if (w0)
    for (int j = lane; j < e_ld; j += 64) {
      const double v = (j < nb) ? u[j] : 0.0;
      if (e64) e64[(size_t)b * e_ld + j] = v;
      if (e32) e32[(size_t)b * e_ld + j] = (float)v;
    }
}

void launch_reduce_solve(bool fp64_part, const void* part, int chunks, int B, int nj, int n,
                         const int* n_use, const double* L, const int* active, double* t_out,
                         double* e64, float* e32, int e_ld, bool solve, hipStream_t s) {
  RB_REQUIRE(nj <= 128 && e_ld <= 128, RB_EUNSUPPORTED, "basis too large for reduce_solve");
  if (fp64_part)
    hipLaunchKernelGGL(k_reduce_solve<double>, dim3(B), dim3(256), 0, s, (const double*)part,
                       chunks, B, nj, n, n_use, L, active, t_out, e64, e32, e_ld, solve ? 1 : 0);
  else
    hipLaunchKernelGGL(k_reduce_solve<float>, dim3(B), dim3(256), 0, s, (const float*)part,
                       chunks, B, nj, n, n_use, L, active, t_out, e64, e32, e_ld, solve ? 1 : 0);
}

// ---- right-hand sides of affine f (eq. 12) ----------------------------------------------
// out[b][pos] = sum_r phi[b][r] f[r][pos] for pos < N, 0 on the padding up to ld.
__global__ void k_combine_rhs(const double* __restrict__ f, int64_t ld, int R,
                              const double* __restrict__ phi, int N, double* __restrict__ out) {
  const int b = blockIdx.y;
  const double* ph = phi + (size_t)b * R;
  for (int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; pos < ld;
       pos += (int64_t)gridDim.x * blockDim.x) {
    double v = 0.0;
    if (pos < N)
      for (int r = 0; r < R; ++r) v += ph[r] * f[(size_t)r * ld + pos];
    out[(size_t)b * ld + pos] = v;
  }
}

void launch_combine_rhs(const double* f, int64_t ld, int R, const double* phi, int B, int N,
                        double* out, hipStream_t s) {
  const int bx = (int)std::min<int64_t>((ld + 255) / 256, 1024);
  hipLaunchKernelGGL(k_combine_rhs, dim3(bx, B), dim3(256), 0, s, f, ld, R, phi, N, out);
}

// ---- active-query list ---------------------------------------------------------------
// qlist[0..cnt) = the b < B with active[b] != 0, in increasing order; qlist[B] = cnt.  One
// block scans the flags 1024 at a time (wave scans with shuffles, then the wave totals).
__global__ __launch_bounds__(1024) void k_compact_active(const int* __restrict__ active, int B,
                                                         int* __restrict__ qlist) {
  __shared__ int wsum[16];
  __shared__ int base;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (threadIdx.x == 0) base = 0;
  __syncthreads();
  for (int c0 = 0; c0 < B; c0 += 1024) {
    const int b = c0 + (int)threadIdx.x;
    const int f = (b < B && active[b]) ? 1 : 0;
    int incl = f;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int v = __shfl_up(incl, d, 64);
      if (lane >= d) incl += v;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    int off = base;
    for (int k = 0; k < w; ++k) off += wsum[k];
    if (f) qlist[off + incl - 1] = b;
    __syncthreads();  // every thread has read base
    if (threadIdx.x == 1023) base = off + incl;
    __syncthreads();
  }
  if (threadIdx.x == 0) qlist[B] = base;
}

void launch_compact_active(const int* active, int B, int* qlist, hipStream_t s) {
  hipLaunchKernelGGL(k_compact_active, dim3(1), dim3(1024), 0, s, active, B, qlist);
}

// ---- CG scalars (Alg. 3) ----------------------------------------------------------------
// Sum of cnt partials by one 256-thread block: four independent loads in flight per
// thread (a one-query RBCG iteration on 255^3, 16 k partials per sum: 1160 -> 1124 us),
// then a fixed tree, so the result does not depend on timing.
__device__ __forceinline__ double sum_parts(const double* p, int cnt, double* sh) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int i = threadIdx.x;
  for (; i + 768 < cnt; i += 1024) {
    s0 += p[i];
    s1 += p[i + 256];
    s2 += p[i + 512];
    s3 += p[i + 768];
  }
  for (; i < cnt; i += 256) s0 += p[i];
  return rbk::block_sum_256((s0 + s1) + (s2 + s3), sh);
}

// Alg. 3, step length: alpha = rho / p^T A p (breakdown if either is not positive)
__global__ __launch_bounds__(256) void k_fin_alpha(const double* __restrict__ part, int stride,
                                                   int cnt, QState q) {
  __shared__ double sh[4];
  const int b = blockIdx.x;
  if (!q.active[b]) return;
  const double pAp = sum_parts(part + (size_t)b * stride, cnt, sh);
  if (threadIdx.x == 0) {
    const double rho = q.rho[b];
    if (!(pAp > 0.0) || !(rho > 0.0)) {
      q.status[b] = RB_EBREAKDOWN;
      q.active[b] = 0;
      q.alpha[b] = 0.0;
    } else {
      q.alpha[b] = rho / pAp;
    }
  }
}

// Alg. 3, stopping test on the recursive residual; flags the query for the true-residual check
__global__ __launch_bounds__(256) void k_fin_rr(const double* __restrict__ part, int stride,
                                                int cnt, QState q, double rtol, int maxit,
                                                int fixed, int defer) {
  __shared__ double sh[4];
  const int b = blockIdx.x;
  if (!q.active[b]) return;
  const double rr = sum_parts(part + (size_t)b * stride, cnt, sh);
  if (threadIdx.x == 0) {
    // an even iteration's x update waits for the next pass B (or a fold); an odd one's
    // pass B applied it
    if (q.apend) q.apend[b] = defer ? q.alpha[b] : 0.0;
    const int it = q.iters[b] + 1;
    q.iters[b] = it;
    const double rel = sqrt(rr / q.fnorm2[b]);
    q.rel_rec[b] = rel;
    if (q.gamma2 > 0.0) {  // adaptive basis size (Sec. 4.1)
      if (q.rr_in[b] < q.gamma2 * rr) q.nuse[b] = min(q.nuse[b] + 1, q.nmax);
      q.rr_in[b] = rr;
    }
    if (fixed) return;
    if (rel <= rtol) {
      q.flag[b] = 1;
    } else if (!(rel == rel)) {
      q.status[b] = RB_EBREAKDOWN;
      q.active[b] = 0;
    } else if (it >= maxit) {
      q.status[b] = RB_ENOCONV;
      q.active[b] = 0;
    }
  }
}

// true residual (eq. relerr): retire on success, else restart with the replaced residual
__global__ __launch_bounds__(256) void k_fin_true(const double* __restrict__ part, int stride,
                                                  int cnt, QState q, double rtol, int maxit,
                                                  const double* __restrict__ part2,
                                                  double floor_factor) {
  __shared__ double sh[4];
  const int b = blockIdx.x;
  if (!q.active[b] || !q.flag[b]) return;
  const double rr = sum_parts(part + (size_t)b * stride, cnt, sh);
  // rounding level of the FP64 residual of x: eps || |A| |x| || (relative to ||f||)
  const double aa = part2 ? sum_parts(part2 + (size_t)b * stride, cnt, sh) : 0.0;
  if (threadIdx.x == 0) {
    const double rel = sqrt(rr / q.fnorm2[b]);
    const double lvl = floor_factor * 0x1p-52 * sqrt(aa / q.fnorm2[b]);
    // The rounding level is a worst-case bound, often far above what the iteration still
    // reaches, so it is accepted only once residual replacements have stopped paying: at
    // two checks in a row the true residual stayed above half of the previous check's (0
    // before the first check).  One such check can be a query that is still converging
    // and was checked just above its tolerance.
    const double prev = q.rel_true[b];
    const bool stalled = prev > 0.0 && rel > 0.5 * prev;
    const int run = stalled ? (q.stalls ? q.stalls[b] + 1 : 2) : 0;
    if (q.stalls) q.stalls[b] = run;
    q.rel_true[b] = rel;
    q.flag[b] = 0;
    if (q.apend) q.apend[b] = 0.0;  // the fold before this check applied it
    if (rel <= rtol || (part2 && run >= 2 && rel <= lvl)) {
      q.active[b] = 0;
      q.status[b] = RB_OK;
      if (q.at_floor && rel > rtol) q.at_floor[b] = 1;
    } else if (q.iters[b] >= maxit) {
      q.active[b] = 0;
      q.status[b] = RB_ENOCONV;
    } else {
      q.restart[b] = 1;
      if (q.gamma2 > 0.0) q.rr_in[b] = rr;  // the replaced residual is preconditioned next
    }
  }
}

// Alg. 3, new direction: rho_new = y^T r (red + black partials); beta (literal or flexible)
__global__ __launch_bounds__(256) void k_fin_beta(const double* __restrict__ pr,
                                                  const double* __restrict__ fr, Segs sg,
                                                  QState q, int flexible) {
  __shared__ double sh[4];
  const int b = blockIdx.x;
  if (!q.active[b]) return;
  // one segment per colour sweep (or one for a whole-vector smoother), in sweep order
  double rho_new = 0.0, x = 0.0;
  for (int c = 0; c < sg.n; ++c) {
    rho_new += sum_parts(pr + sg.off[c] + (size_t)b * sg.cnt[c], sg.cnt[c], sh);
    if (flexible && fr) x += sum_parts(fr + sg.off[c] + (size_t)b * sg.cnt[c], sg.cnt[c], sh);
  }
  if (threadIdx.x == 0) {
    const double rho_old = q.rho[b];
    double beta;
    if (q.restart[b]) {
      beta = 0.0;
      q.restart[b] = 0;
    } else if (flexible) {
      beta = (rho_new - x) / rho_old;
    } else {
      beta = rho_new / rho_old;
    }
    q.beta[b] = beta;
    q.rho[b] = rho_new;
  }
}

// ||f||^2 per query (RBCG init) or ||r||^2 (RBI loop) from partials
__global__ __launch_bounds__(256) void k_fin_sum(const double* __restrict__ part, int stride,
                                                 int cnt, double* __restrict__ out,
                                                 const int* __restrict__ active) {
  __shared__ double sh[4];
  const int b = blockIdx.x;
  if (active && !active[b]) return;
  const double s = sum_parts(part + (size_t)b * stride, cnt, sh);
  if (threadIdx.x == 0) out[b] = s;
}

void launch_fin_alpha(const double* part, int stride, int cnt, const QState& q, int B,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_fin_alpha, dim3(B), dim3(256), 0, s, part, stride, cnt, q);
}
void launch_fin_rr(const double* part, int stride, int cnt, const QState& q, int B, double rtol,
                   int maxit, bool fixed, hipStream_t s, bool defer) {
  hipLaunchKernelGGL(k_fin_rr, dim3(B), dim3(256), 0, s, part, stride, cnt, q, rtol, maxit,
                     fixed ? 1 : 0, defer ? 1 : 0);
}
void launch_fin_true(const double* part, int stride, int cnt, const QState& q, int B, double rtol,
                     int maxit, hipStream_t s, const double* part2, double floor_factor) {
  hipLaunchKernelGGL(k_fin_true, dim3(B), dim3(256), 0, s, part, stride, cnt, q, rtol, maxit,
                     part2, floor_factor);
}
void launch_fin_beta(const double* pr, const double* fr, const Segs& sg, const QState& q, int B,
                     bool flexible, hipStream_t s) {
  hipLaunchKernelGGL(k_fin_beta, dim3(B), dim3(256), 0, s, pr, fr, sg, q, flexible ? 1 : 0);
}
void launch_fin_sum(const double* part, int stride, int cnt, double* out, const int* active,
                    int B, hipStream_t s) {
  hipLaunchKernelGGL(k_fin_sum, dim3(B), dim3(256), 0, s, part, stride, cnt, out, active);
}

// ---- small helpers ---------------------------------------------------------------------
// Correction folding of the CG iterate: x_b += xc_b, xc_b = 0 for the flagged queries.
// Rows are ld (a multiple of 64) doubles; padding is zero in both vectors.  Every block
// takes a slice of every flagged row (few rows are flagged at a time: each query reaches
// its true-residual check once or twice), so a flagged row is folded by the whole grid.
// A pending update (apend[b] != 0, direction p_b) joins the correction first, as pass B
// would have added it: x_b += (xc_b + apend[b] p_b).
__global__ __launch_bounds__(256) void k_fold(const int* __restrict__ flag, int B,
                                              double2* __restrict__ x, double2* __restrict__ xc,
                                              int64_t ld2, int64_t slice,
                                              const double* __restrict__ apend,
                                              const double2* __restrict__ p) {
  const int64_t i0 = (int64_t)blockIdx.x * slice;
  const int64_t i1 = i0 + slice < ld2 ? i0 + slice : ld2;
  for (int b = 0; b < B; ++b) {
    if (flag && !flag[b]) continue;  // uniform across the block
    double2* xb = x + (size_t)b * ld2;
    double2* cb = xc + (size_t)b * ld2;
    const double ap = apend ? apend[b] : 0.0;
    if (ap != 0.0) {
      const double2* pb = p + (size_t)b * ld2;
      for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
        const double2 a = xb[i], c = cb[i], v = pb[i];
        xb[i] = make_double2(a.x + (c.x + ap * v.x), a.y + (c.y + ap * v.y));
        cb[i] = make_double2(0.0, 0.0);
      }
    } else {
      for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
        const double2 a = xb[i], c = cb[i];
        xb[i] = make_double2(a.x + c.x, a.y + c.y);
        cb[i] = make_double2(0.0, 0.0);
      }
    }
  }
}
void launch_fold(const int* flag, int B, double* x, double* xc, int64_t ld, hipStream_t s,
                 const double* apend, const double* p) {
  if (B <= 0) return;
  RB_REQUIRE(!apend || p, RB_EINVAL, "fold: a pending update needs its direction");
  const int64_t ld2 = ld / 2;
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(1024, (ld2 + 255) / 256));
  const int64_t slice = (ld2 + blocks - 1) / blocks;
  hipLaunchKernelGGL(k_fold, dim3(blocks), dim3(256), 0, s, flag, B, (double2*)x, (double2*)xc,
                     ld2, slice, apend, (const double2*)p);
}

// dst[b][pos] = value for pos < n (fill kernel; graph-safe replacement for memset)
template <typename T>
__global__ void k_fill(T* __restrict__ dst, int64_t ld, int64_t n, T value) {
  const int b = blockIdx.y;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[(size_t)b * ld + i] = value;
}
template <typename T>
void launch_fill(T* dst, int64_t ld, int64_t n, int B, T value, hipStream_t s) {
  int bx = (int)((n + 255) / 256);
  if (bx > 2048) bx = 2048;
  if (bx < 1) bx = 1;
  hipLaunchKernelGGL(k_fill<T>, dim3(bx, B), dim3(256), 0, s, dst, ld, n, value);
}
template void launch_fill<double>(double*, int64_t, int64_t, int, double, hipStream_t);
template void launch_fill<float>(float*, int64_t, int64_t, int, float, hipStream_t);
template void launch_fill<int>(int*, int64_t, int64_t, int, int, hipStream_t);

// r_b = phi_b * f[pos] (shared term) and partial ||r_b||^2
__global__ __launch_bounds__(256) void k_init_rhs(const double* __restrict__ f, int64_t f_ld,
                                                  const double* __restrict__ scale, int N,
                                                  double* __restrict__ r, int64_t ld,
                                                  double* __restrict__ part, int per_thread,
                                                  float* __restrict__ r32) {
  __shared__ double sh[4];
  const int b = blockIdx.y;
  const double sc = scale[b];
  const double* fb = f + (size_t)b * f_ld;
  double acc = 0.0;
  const int base = blockIdx.x * 256 * per_thread;
  for (int t = 0; t < per_thread; ++t) {
    const int pos = base + t * 256 + threadIdx.x;
    if (pos >= N) break;
    const double v = sc * fb[pos];
    r[(size_t)b * ld + pos] = v;
    if (r32) r32[(size_t)b * ld + pos] = (float)v;
    acc += v * v;
  }
  const double s = rbk::block_sum_256(acc, sh);
  if (threadIdx.x == 0) part[(size_t)b * gridDim.x + blockIdx.x] = s;
}
int launch_init_rhs(const double* f, int64_t f_ld, const double* scale, int N, double* r,
                    int64_t ld, int B, double* part, int per_thread, hipStream_t s, float* r32) {
  const int chunks = (N + 256 * per_thread - 1) / (256 * per_thread);
  hipLaunchKernelGGL(k_init_rhs, dim3(chunks, B), dim3(256), 0, s, f, f_ld, scale, N, r, ld, part,
                     per_thread, r32);
  return chunks;
}

// precision shadows of the basis (round to nearest even)
__global__ void k_cast_f32(const double* __restrict__ src, float* __restrict__ dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (float)src[i];
}
__global__ void k_cast_bf16(const double* __restrict__ src, uint16_t* __restrict__ dst,
                            int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = rbk::f32_to_bf16_rne((float)src[i]);
}
__global__ void k_widen(const float* __restrict__ src, double* __restrict__ dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (double)src[i];
}
void launch_widen(const float* src, double* dst, int64_t n, hipStream_t s) {
  int bx = (int)((n + 255) / 256);
  if (bx > 8192) bx = 8192;
  if (bx < 1) bx = 1;
  hipLaunchKernelGGL(k_widen, dim3(bx), dim3(256), 0, s, src, dst, n);
}

void launch_cast(const double* src, void* dst, int64_t n, rb_prec prec, hipStream_t s) {
  int bx = (int)((n + 255) / 256);
  if (bx > 8192) bx = 8192;
  if (prec == RB_PREC_FP32)
    hipLaunchKernelGGL(k_cast_f32, dim3(bx), dim3(256), 0, s, src, (float*)dst, n);
  else
    hipLaunchKernelGGL(k_cast_bf16, dim3(bx), dim3(256), 0, s, src, (uint16_t*)dst, n);
}

}  // namespace rb
