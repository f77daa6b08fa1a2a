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

// Accumulate a 64x64 tile:  acc += A(i, k) * B(k, j) for i in [0, M), j in
// [0, N) (tile-local), k in [k0, k1).  A(i, k) = A[i*ars + k*acs],
// B(k, j) = B[k*brs + j*bcs].  256 threads; thread (tx, ty) = (tid % 16,
// tid / 16) owns rows ty + 16*ii and columns tx + 16*jj (ii, jj < 4).
// Staging is coalesced along whichever stride is 1.  sA, sB: LDS [KT*TILE].
__device__ inline void tile_gemm_acc(double acc[4][4], const double *__restrict__ A, long ars, long acs,
                                     const double *__restrict__ B, long brs, long bcs, int M, int N, int k0,
                                     int k1, double *sA, double *sB) {
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  const bool a_rowfast = (ars == 1);
  const bool b_colfast = (bcs == 1);
  for (int kb = k0; kb < k1; kb += KT) {
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
      double v = 0.0;
      if (i < M && kk < k1) v = A[(long)i * ars + (long)kk * acs];
      sA[k * TILE + i] = v;
      int j;
      if (b_colfast) {
        j = e & 63;
        k = e >> 6;
      } else {
        k = e & 15;
        j = e >> 4;
      }
      kk = kb + k;
      v = 0.0;
      if (j < N && kk < k1) v = B[(long)kk * brs + (long)j * bcs];
      sB[k * TILE + j] = v;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < KT; ++k) {
      double a[4], b[4];
#pragma unroll
      for (int ii = 0; ii < 4; ++ii) a[ii] = sA[k * TILE + ty + 16 * ii];
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) b[jj] = sB[k * TILE + tx + 16 * jj];
#pragma unroll
      for (int ii = 0; ii < 4; ++ii)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) acc[ii][jj] = fma(a[ii], b[jj], acc[ii][jj]);
    }
    __syncthreads();
  }
}

__device__ inline void tile_zero(double acc[4][4]) {
#pragma unroll
  for (int ii = 0; ii < 4; ++ii)
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) acc[ii][jj] = 0.0;
}

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
