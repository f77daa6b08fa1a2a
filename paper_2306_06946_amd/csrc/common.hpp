// Device-side helpers shared by the library's kernels: error checking, the
// FP64 LDS-tiled GEMM tile used by the supernodal factor and solves.
#pragma once

#include <hip/hip_runtime.h>

#include <stdexcept>
#include <string>

#include "icr_internal.hpp"

namespace icr {

struct HipError : std::runtime_error {
  hipError_t code;
  HipError(hipError_t c, const std::string &where)
      : std::runtime_error(where + ": " + hipGetErrorString(c)), code(c) {}
};

#define ICR_HIP(call)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess) throw ::icr::HipError(e_, std::string(#call) + " @" + __FILE__ + \
                                                   ":" + std::to_string(__LINE__));     \
  } while (0)

#define ICR_LAUNCH_CHECK() ICR_HIP(hipGetLastError())

constexpr int TILE = 64;   // output tile edge of the FP64 GEMM tiles
constexpr int KT = 16;     // K-chunk staged in LDS per iteration

// ---------------------------------------------------------------------------
// 64x64 FP64 MFMA tile accumulators.  Each exposes for_each(f) visiting the
// tile-local (i, j) of every value the calling thread owns.
// ---------------------------------------------------------------------------

typedef double mfma_d4 __attribute__((ext_vector_type(4)));

// MFMA layout (v_mfma_f64_16x16x4f64, checked on gfx950): A(i, k) comes from
// lane i + 16 k, B(k, j) from lane j + 16 k, and D(i, j) lands in lane
// j + 16 (i % 4), register i / 4.  Wave w owns the 32x32 quadrant
// (32 (w >> 1), 32 (w & 1)) as 2x2 blocks of 16x16.
struct AccM {
  mfma_d4 c[2][2];
  __device__ void zero() {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) c[a][b] = mfma_d4{0.0, 0.0, 0.0, 0.0};
  }
  __device__ void acc(const double *A, long ars, long acs, const double *B, long brs, long bcs, int M, int N, int k0,
                      int k1, double *sA, double *sB);
  template <class F>
  __device__ void for_each(F &&f) {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int r0 = 32 * (w >> 1), c0 = 32 * (w & 1);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int t = 0; t < 4; ++t) f(r0 + 16 * a + 4 * t + (l >> 4), c0 + 16 * b + (l & 15), c[a][b][t]);
  }
};

// Register-prefetched staging: the next K-chunk is fetched from global memory
// into registers while the MFMAs of the current chunk run from LDS.
__device__ inline void load_chunk_regs(const double *__restrict__ A, long ars, long acs, const double *__restrict__ B,
                                       long brs, long bcs, int M, int N, int kb, int k1, double ra[4],
                                       double rb[4]) {
  const int tid = threadIdx.x;
  const bool a_rowfast = (ars == 1);
  const bool b_colfast = (bcs == 1);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    int e = tid + 256 * q;
    int i, k;
    if (a_rowfast) {
      i = e & 63;
      k = e >> 6;
    } else {
      k = e & 15;
      i = e >> 4;
    }
    int kk = kb + k;
    ra[q] = (i < M && kk < k1) ? A[(long)i * ars + (long)kk * acs] : 0.0;
    int j;
    if (b_colfast) {
      j = e & 63;
      k = e >> 6;
    } else {
      k = e & 15;
      j = e >> 4;
    }
    kk = kb + k;
    rb[q] = (j < N && kk < k1) ? B[(long)kk * brs + (long)j * bcs] : 0.0;
  }
}

__device__ inline void store_chunk_lds(bool a_rowfast, bool b_colfast, const double ra[4], const double rb[4],
                                       double *sA, double *sB) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    int e = tid + 256 * q;
    int i, k;
    if (a_rowfast) {
      i = e & 63;
      k = e >> 6;
    } else {
      k = e & 15;
      i = e >> 4;
    }
    sA[k * TILE + i] = ra[q];
    int j;
    if (b_colfast) {
      j = e & 63;
      k = e >> 6;
    } else {
      k = e & 15;
      j = e >> 4;
    }
    sB[k * TILE + j] = rb[q];
  }
}

__device__ inline void AccM::acc(const double *A, long ars, long acs, const double *B, long brs, long bcs, int M,
                                 int N, int k0, int k1, double *sA, double *sB) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int r0 = 32 * (w >> 1), c0 = 32 * (w & 1);
  const int li = l & 15, lk = l >> 4;
  const bool a_rowfast = (ars == 1), b_colfast = (bcs == 1);
  if (k0 >= k1) return;
  double ra[4], rb[4];
  load_chunk_regs(A, ars, acs, B, brs, bcs, M, N, k0, k1, ra, rb);
  for (int kb = k0; kb < k1; kb += KT) {
    store_chunk_lds(a_rowfast, b_colfast, ra, rb, sA, sB);
    __syncthreads();
    if (kb + KT < k1) load_chunk_regs(A, ars, acs, B, brs, bcs, M, N, kb + KT, k1, ra, rb);
#pragma unroll
    for (int kk = 0; kk < KT; kk += 4) {
      const int k = kk + lk;
      double a0 = sA[k * TILE + r0 + li], a1 = sA[k * TILE + r0 + 16 + li];
      double b0 = sB[k * TILE + c0 + li], b1 = sB[k * TILE + c0 + 16 + li];
      c[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, c[0][0], 0, 0, 0);
      c[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, c[0][1], 0, 0, 0);
      c[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, c[1][0], 0, 0, 0);
      c[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, c[1][1], 0, 0, 0);
    }
    __syncthreads();
  }
}

typedef float mfma_f4 __attribute__((ext_vector_type(4)));

// One 16x16x4 MFMA per element type: FP64 (v_mfma_f64_16x16x4f64) or FP32
// (v_mfma_f32_16x16x4f32).  Both take A(i, k) from lane i + 16 k and B(k, j)
// from lane j + 16 k; they differ in where D(i, j) lands (checked on gfx950):
// FP64 in lane j + 16 (i % 4), register i / 4; FP32 in lane j + 16 (i / 4),
// register i % 4.
template <class T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef mfma_d4 V;
  __device__ static V op(double a, double b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static int row(int lane, int r) { return 4 * r + (lane >> 4); }
};
template <>
struct Mfma<float> {
  typedef mfma_f4 V;
  __device__ static V op(float a, float b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// Generalised MFMA tile: 4 waves as 2x2, each (16 WB) x (16 WB) of 16x16
// blocks, output tile T = 32 WB, element type E (double or float, operands
// and accumulation alike).  The K-chunk of A (T x KC) and B (KC x T) is
// staged in LDS as [k][i] / [k][j] rows padded to T + 1 elements (no bank
// conflicts for either staging order or the MFMA operand reads), the next
// chunk is prefetched into registers while the MFMAs of the current one run.
template <int WB, int KC = KT, class E = double>
struct AccMT {
  typedef E elem;
  typedef typename Mfma<E>::V V;
  static constexpr int T = 32 * WB;
  static constexpr int TP = T + 1;
  static constexpr int NE = T * KC / 256;   // staged elements per thread and operand
  static constexpr int LDS = 2 * KC * TP;   // elements of LDS
  V c[WB][WB];
  __device__ void zero() {
#pragma unroll
    for (int a = 0; a < WB; ++a)
#pragma unroll
      for (int b = 0; b < WB; ++b) c[a][b] = V{0, 0, 0, 0};
  }
  // Thread tid stages, for every q < NE, element (i, k) of A: with rows
  // contiguous (AF) i = tid % T, k = tid / T + q (256 / T); else k = tid % KC,
  // i = tid / KC + (256 / KC) q; likewise (k, j) of B with BF.  One base pointer per
  // operand and a constant stride per q.
  // c += A(i, k) B(k, j) over k in [k0, k1); A(i, k) = A[i ars + k acs],
  // B(k, j) = B[k brs + j bcs]; rows i < M and columns j < N of the tile.
  // TRI: A is lower triangular, A(i, k) = 0 for k > i + tri.
  template <bool AF, bool BF, bool TRI = false>
  __device__ void acc(const E *A, long ars, long acs, const E *B, long brs, long bcs, int M, int N, int k0, int k1,
                      E *lds, int tri = 0) {
    const int tid = threadIdx.x;
    const int w = tid >> 6, l = tid & 63;
    const int r0 = (T / 2) * (w >> 1), c0 = (T / 2) * (w & 1);
    const int li = l & 15, lk = l >> 4;
    if (k0 >= k1) return;
    constexpr int QS = 256 / T;    // k step per q when rows are contiguous
    constexpr int QK = 256 / KC;   // row step per q when k is contiguous
    const int ia = AF ? tid % T : tid / KC, ka = AF ? tid / T : tid % KC;
    const int jb = BF ? tid % T : tid / KC, kbb = BF ? tid / T : tid % KC;
    const long qa = AF ? QS * acs : QK * ars, qb = BF ? QS * brs : QK * bcs;
    const E *pa = A + (long)ia * ars + (long)(k0 + ka) * acs;
    const E *pb = B + (long)(k0 + kbb) * brs + (long)jb * bcs;
    E *sa = lds + ka * TP + ia, *sb = lds + KC * TP + kbb * TP + jb;
    const int sqa = AF ? QS * TP : QK, sqb = BF ? QS * TP : QK;
    E ra[NE], rb[NE];
    auto load = [&](int kb) {
#pragma unroll
      for (int q = 0; q < NE; ++q) {
        const int i = AF ? ia : ia + QK * q, k = kb + (AF ? ka + QS * q : ka);
        ra[q] = (i < M && k < k1 && (!TRI || k <= i + tri)) ? pa[q * qa] : E(0);
        const int j = BF ? jb : jb + QK * q, kq = kb + (BF ? kbb + QS * q : kbb);
        rb[q] = (j < N && kq < k1) ? pb[q * qb] : E(0);
      }
    };
    load(k0);
    for (int kb = k0; kb < k1; kb += KC) {
#pragma unroll
      for (int q = 0; q < NE; ++q) {
        sa[q * sqa] = ra[q];
        sb[q * sqb] = rb[q];
      }
      __syncthreads();
      if (kb + KC < k1) {
        pa += KC * acs;
        pb += KC * brs;
        load(kb + KC);
      }
#pragma unroll
      for (int kk = 0; kk < KC; kk += 4) {
        const int k = kk + lk;
        E av[WB], bv[WB];
#pragma unroll
        for (int a = 0; a < WB; ++a) av[a] = lds[k * TP + r0 + 16 * a + li];
#pragma unroll
        for (int b = 0; b < WB; ++b) bv[b] = lds[KC * TP + k * TP + c0 + 16 * b + li];
#pragma unroll
        for (int a = 0; a < WB; ++a)
#pragma unroll
          for (int b = 0; b < WB; ++b) c[a][b] = Mfma<E>::op(av[a], bv[b], c[a][b]);
      }
      __syncthreads();
    }
  }
  template <class F>
  __device__ void for_each(F &&f) {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int r0 = (T / 2) * (w >> 1), c0 = (T / 2) * (w & 1);
#pragma unroll
    for (int a = 0; a < WB; ++a)
#pragma unroll
      for (int b = 0; b < WB; ++b)
#pragma unroll
        for (int t = 0; t < 4; ++t) f(r0 + 16 * a + Mfma<E>::row(l, t), c0 + 16 * b + (l & 15), c[a][b][t]);
  }
};
typedef AccMT<2, 32> AccS;          // 64 x 64 FP64, K-chunk 32
typedef AccMT<2, 32, float> AccS32;  // 64 x 64 FP32, K-chunk 32

// The tile accumulator of the factor kernels.
typedef AccM Acc;


// Lower-triangle tile index x -> (I, J), I >= J, row-major over the triangle.
__device__ inline void tri_index(int x, int &I, int &J) {
  int i = (int)((sqrt(8.0 * (double)x + 1.0) - 1.0) * 0.5);
  while ((i + 1) * (i + 2) / 2 <= x) ++i;
  while (i * (i + 1) / 2 > x) --i;
  I = i;
  J = x - i * (i + 1) / 2;
}

inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

}  // namespace icr
