// Supernodal (multifrontal) FP64 Cholesky of A on the device: the factor the
// multi-RHS solves of W_H = H A^-1 H^T run against (Eq. 28).
//
// Fronts are processed by height level of the dissection tree, bottom-up.  A
// level's fronts are assembled together (children's Schur complements pulled
// through index maps, then A's blocks scattered), then partially factored by a
// right-looking blocked Cholesky over 64-column steps (diagonal tile
// factor + inverse, panel solve, trailing update), all fronts of the level in
// the same launches.  Finally each supernode's diagonal block inverse
// L_ss^{-1} is formed (used by the solves as a dense product).
#include <algorithm>
#include <cmath>

#include "scene.hpp"

namespace icr {

namespace {

// Zero the front and pull every child's update matrix (its trailing Schur
// complement) through the child's index map.  One front per blockIdx.y.
__global__ void k_front_init(const SupDev *__restrict__ sup, const int *__restrict__ level_sup,
                             const int *__restrict__ child, const int *__restrict__ invmap_off,
                             const int *__restrict__ invmap, double *__restrict__ front) {
  const SupDev S = sup[level_sup[blockIdx.y]];
  const int f = 3 * (S.ncol + S.nb);
  const long total = (long)f * f;
  double *F = front + S.front_off;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    int i = (int)(e % f), j = (int)(e / f);
    double v = 0.0;
    if (i >= j) {
      for (int c = 0; c < S.nchild; ++c) {
        const int ch = child[S.child_off + c];
        const int *inv = invmap + invmap_off[S.child_off + c];
        int ii = inv[i / 3], jj = inv[j / 3];
        if (ii >= 0 && jj >= 0) {
          const SupDev C = sup[ch];
          const int fc = 3 * (C.ncol + C.nb), n3c = 3 * C.ncol;
          v += front[C.front_off + (long)(n3c + 3 * ii + i % 3) + (long)(n3c + 3 * jj + j % 3) * fc];
        }
      }
    }
    F[e] = v;
  }
}

__global__ void k_front_add_A(const AScatter *__restrict__ list, int count, const SupDev *__restrict__ sup,
                              const double *__restrict__ Ab, double *__restrict__ front) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  AScatter a = list[e];
  const SupDev S = sup[a.s];
  const int f = 3 * (S.ncol + S.nb);
  double *F = front + S.front_off;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) F[(long)(3 * a.lr + i) + (long)(3 * a.lc + j) * f] += Ab[9L * a.blk + 3 * i + j];
}

// Factor the t x t diagonal tile at column k of every front of the level, and
// write its inverse into the diagonal tile of L_ss^{-1} (upper part zero).
__global__ __launch_bounds__(256) void k_potrf_tile(const SupDev *__restrict__ sup,
                                                    const int *__restrict__ level_sup, int k,
                                                    double *__restrict__ front, double *__restrict__ linv,
                                                    int *__restrict__ err) {
  __shared__ double D[64][64];
  __shared__ double X[64][64];
  const SupDev S = sup[level_sup[blockIdx.x]];
  const int n3 = 3 * S.ncol, f = 3 * (S.ncol + S.nb);
  if (k >= n3) return;
  const int t = min(64, n3 - k);
  double *F = front + S.front_off;
  const int tid = threadIdx.x;
  for (int e = tid; e < t * t; e += 256) {
    int i = e % t, j = e / t;
    D[i][j] = (i >= j) ? F[(long)(k + i) + (long)(k + j) * f] : 0.0;
  }
  __syncthreads();
  for (int c = 0; c < t; ++c) {
    if (tid == 0) {
      double d = D[c][c];
      if (!(d > 0.0)) {
        atomicMin(err, 3 * S.col0 + k + c);
        d = 1.0;
      }
      D[c][c] = sqrt(d);
    }
    __syncthreads();
    for (int i = c + 1 + tid; i < t; i += 256) D[i][c] = D[i][c] / D[c][c];
    __syncthreads();
    const int rem = t - c - 1;
    for (int e = tid; e < rem * rem; e += 256) {
      int i = c + 1 + e % rem, j = c + 1 + e / rem;
      if (i >= j) D[i][j] -= D[i][c] * D[j][c];
    }
    __syncthreads();
  }
  for (int e = tid; e < t * t; e += 256) {
    int i = e % t, j = e / t;
    if (i >= j) F[(long)(k + i) + (long)(k + j) * f] = D[i][j];
  }
  // inverse of the lower-triangular tile, one column per thread
  if (tid < t) {
    const int j = tid;
    for (int i = 0; i < j; ++i) X[i][j] = 0.0;
    for (int i = j; i < t; ++i) {
      double s = (i == j) ? 1.0 : 0.0;
      for (int q = j; q < i; ++q) s -= D[i][q] * X[q][j];
      X[i][j] = s / D[i][i];
    }
  }
  __syncthreads();
  double *Li = linv + S.linv_off;
  for (int e = tid; e < t * t; e += 256) {
    int i = e % t, j = e / t;
    Li[(long)(k + i) + (long)(k + j) * n3] = X[i][j];
  }
}

// Panel rows below the diagonal tile: P <- P * D^{-T}.
__global__ __launch_bounds__(256) void k_trsm_panel(const SupDev *__restrict__ sup,
                                                    const int *__restrict__ level_sup, int k,
                                                    double *__restrict__ front, const double *__restrict__ linv) {
  __shared__ double sA[KT * TILE], sB[KT * TILE];
  const SupDev S = sup[level_sup[blockIdx.y]];
  const int n3 = 3 * S.ncol, f = 3 * (S.ncol + S.nb);
  if (k >= n3) return;
  const int t = min(64, n3 - k);
  const int i0 = k + t + TILE * blockIdx.x;
  if (i0 >= f) return;
  const int M = min(TILE, f - i0);
  double *F = front + S.front_off;
  const double *Di = linv + S.linv_off + k + (long)k * n3;
  Acc acc;
  acc.zero();
  // out(i, j) = sum_c P(i, c) * Dinv(j, c)
  acc.acc(F + i0 + (long)k * f, 1, f, Di, n3, 1, M, t, 0, t, sA, sB);
  acc.for_each([&](int i, int j, double v) {
    if (i < M && j < t) F[(long)(i0 + i) + (long)(k + j) * f] = v;
  });
}

// Trailing update of the lower triangle: F(i, j) -= sum_c P(i, c) P(j, c).
__global__ __launch_bounds__(256) void k_trailing(const SupDev *__restrict__ sup, const int *__restrict__ level_sup,
                                                  int k, double *__restrict__ front) {
  __shared__ double sA[KT * TILE], sB[KT * TILE];
  const SupDev S = sup[level_sup[blockIdx.y]];
  const int n3 = 3 * S.ncol, f = 3 * (S.ncol + S.nb);
  if (k >= n3) return;
  const int t = min(64, n3 - k);
  const int base = k + t;
  const int rem = f - base;
  if (rem <= 0) return;
  const int nt = (rem + TILE - 1) / TILE;
  if ((int)blockIdx.x >= nt * (nt + 1) / 2) return;
  int I, J;
  tri_index(blockIdx.x, I, J);
  const int i0 = base + TILE * I, j0 = base + TILE * J;
  const int M = min(TILE, f - i0), N = min(TILE, f - j0);
  double *F = front + S.front_off;
  Acc acc;
  acc.zero();
  acc.acc(F + i0 + (long)k * f, 1, f, F + j0 + (long)k * f, f, 1, M, N, 0, t, sA, sB);
  acc.for_each([&](int i, int j, double v) {
    if (i < M && j < N) F[(long)(i0 + i) + (long)(j0 + j) * f] -= v;
  });
}

// L_ss^{-1}: one workgroup per 64-column tile J, marching down tile rows:
// X(I, J) = -D_I^{-1} * sum_{K=J}^{I-1} L(I, K) X(K, J),  X(J, J) = D_J^{-1}.
__global__ __launch_bounds__(256) void k_linv(const SupDev *__restrict__ sup, const int *__restrict__ level_sup,
                                              const double *__restrict__ front, double *__restrict__ linv) {
  __shared__ double sA[KT * TILE], sB[KT * TILE];
  __shared__ double Sx[TILE * TILE];
  const SupDev S = sup[level_sup[blockIdx.y]];
  const int n3 = 3 * S.ncol, f = 3 * (S.ncol + S.nb);
  const int ntl = (n3 + TILE - 1) / TILE;
  const int J = blockIdx.x;
  if (J >= ntl) return;
  const double *F = front + S.front_off;
  double *X = linv + S.linv_off;
  const int j0 = TILE * J, N = min(TILE, n3 - j0);
  for (int I = J + 1; I < ntl; ++I) {
    const int i0 = TILE * I, M = min(TILE, n3 - i0);
    Acc acc;
    acc.zero();
    acc.acc(F + i0, 1, f, X + j0 * (long)n3, 1, n3, M, N, j0, i0, sA, sB);
    // stage S = acc in LDS (column-major 64x64)
    acc.for_each([&](int i, int j, double v) { Sx[i + TILE * j] = v; });
    __syncthreads();
    Acc out;
    out.zero();
    out.acc(X + i0 + (long)i0 * n3, 1, n3, Sx, 1, TILE, M, N, 0, M, sA, sB);
    out.for_each([&](int i, int j, double v) {
      if (i < M && j < N) X[(long)(i0 + i) + (long)(j0 + j) * n3] = -v;
    });
    __threadfence_block();
    __syncthreads();
  }
  // zero the strictly-upper tiles of this column tile (never read, kept clean)
  for (int I = 0; I < J; ++I) {
    const int i0 = TILE * I;
    for (int e = threadIdx.x; e < TILE * N; e += 256) {
      int i = e % TILE, j = e / TILE;
      X[(long)(i0 + i) + (long)(j0 + j) * n3] = 0.0;
    }
  }
}

}  // namespace

void run_numeric_factor(icr_scene *s) {
  auto &F = s->fac;
  auto &m = s->mesh;
  hipStream_t st = s->stream;
  ICR_HIP(hipMemsetAsync(F.d_err, 0x7f, sizeof(int), st));
  hipEvent_t e0, e1;
  ICR_HIP(hipEventCreate(&e0));
  ICR_HIP(hipEventCreate(&e1));
  ICR_HIP(hipEventRecord(e0, st));
  for (size_t l = 0; l < F.levels.size(); ++l) {
    const LevelInfo &L = F.levels[l];
    if (L.count == 0) continue;
    const int *lsup = F.d_level_sup + L.first;
    int gx = (int)std::min<long long>(1024, (L.max_f2 + 255) / 256);
    k_front_init<<<dim3(gx, L.count), 256, 0, st>>>(F.d_sup, lsup, F.d_child, F.d_invmap_off, F.d_invmap,
                                                    F.d_front);
    ICR_LAUNCH_CHECK();
    if (L.a_count > 0) {
      k_front_add_A<<<cdiv(L.a_count, 256), 256, 0, st>>>(F.d_ascat + L.a_first, L.a_count, F.d_sup, m.d_A,
                                                          F.d_front);
      ICR_LAUNCH_CHECK();
    }
    for (int k = 0; k < L.max_n3; k += TILE) {
      k_potrf_tile<<<L.count, 256, 0, st>>>(F.d_sup, lsup, k, F.d_front, F.d_linv, F.d_err);
      ICR_LAUNCH_CHECK();
      int rem = L.max_f3 - k;   // upper bound of rows below the diagonal tile (+t)
      int pt = cdiv(std::max(rem, 1), TILE);
      k_trsm_panel<<<dim3(pt, L.count), 256, 0, st>>>(F.d_sup, lsup, k, F.d_front, F.d_linv);
      ICR_LAUNCH_CHECK();
      k_trailing<<<dim3(pt * (pt + 1) / 2, L.count), 256, 0, st>>>(F.d_sup, lsup, k, F.d_front);
      ICR_LAUNCH_CHECK();
    }
    k_linv<<<dim3(std::max(1, L.max_rows_tiles), L.count), 256, 0, st>>>(F.d_sup, lsup, F.d_front, F.d_linv);
    ICR_LAUNCH_CHECK();
  }
  ICR_HIP(hipEventRecord(e1, st));
  ICR_HIP(hipEventSynchronize(e1));
  float ms = 0;
  ICR_HIP(hipEventElapsedTime(&ms, e0, e1));
  F.ms = ms;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}

}  // namespace icr
