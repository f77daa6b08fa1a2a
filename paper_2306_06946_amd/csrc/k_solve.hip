// Solves against the supernodal factor P A P^T = L L^T.
//
// Multi-RHS (W_H = H A^-1 H^T, Eq. 28): with Z = L^{-1} P H^T,
// W_H = Z^T Z.  Contacts are sorted by the postorder index of the supernode
// holding their node, so the contacts below supernode s form one contiguous
// range [lo_s, hi_s) and its RHS front X_s has 3 (hi_s - lo_s) columns.  Per
// height level, bottom-up:
//   X_s  = unit columns of its own contacts + children's updates (pulled)
//   Z_s  = L_ss^{-1} X_s[:n_s]                   (triangular dense product)
//   X_s[n_s:] -= L_21 Z_s                        (update passed to the parent)
//   Wp[range_s, range_s] += Z_s^T Z_s            (lower tiles; ranges of one
//                                                 level are disjoint)
// then W_H is read out of Wp in contact order (exactly symmetric).
//
// Single RHS (free motion, corrective motion): the same forward sweep with one
// dense column, then the backward sweep top-down
//   x_s = L_ss^{-T} (y_s - L_21^T x[below rows of s]).
#include <algorithm>

#include "scene.hpp"

namespace icr {

namespace {

// ---- contact ordering -------------------------------------------------------

// Sort the contacts by (supernode, node, index) with a bitonic network on a
// packed 64-bit key.  Invalid ids (out of range, clamped) get the key nsup,
// outside every supernode range, and duplicates are flagged; both make the
// call fail on the host.
__global__ __launch_bounds__(1024) void k_sort_contacts(int nc, int N, int nsup, const int *__restrict__ node_ids,
                                                        const int *__restrict__ sup_of_node,
                                                        const uint8_t *__restrict__ fixed,
                                                        int *__restrict__ keys_sorted, int *__restrict__ order,
                                                        int *__restrict__ pos, int *__restrict__ cerr) {
  __shared__ unsigned long long kv[8192];
  int n2 = 1;
  while (n2 < nc) n2 <<= 1;
  for (int i = threadIdx.x; i < n2; i += blockDim.x) {
    unsigned long long v = ~0ull;
    if (i < nc) {
      int node = node_ids[i];
      unsigned long long key = (unsigned long long)nsup, nd = 0;
      if (node < 0 || node >= N || fixed[node]) {
        atomicMax(cerr, 1);
      } else {
        key = (unsigned long long)sup_of_node[node];
        nd = (unsigned long long)node;
      }
      v = (key << 37) | (nd << 13) | (unsigned long long)i;
    }
    kv[i] = v;
  }
  __syncthreads();
  for (int k = 2; k <= n2; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < n2; i += blockDim.x) {
        int l = i ^ j;
        if (l > i) {
          unsigned long long a = kv[i], b = kv[l];
          bool up = ((i & k) == 0);
          if ((a > b) == up) {
            kv[i] = b;
            kv[l] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int p = threadIdx.x; p < nc; p += blockDim.x) {
    unsigned long long v = kv[p];
    int c = (int)(v & 0x1fffull);
    order[p] = c;
    keys_sorted[p] = (int)(v >> 37);
    pos[c] = p;
    if (p > 0 && (kv[p - 1] >> 13) == (v >> 13) && (int)(v >> 37) < nsup) atomicMax(cerr, 2);
  }
}

__device__ inline int lower_bound_i(const int *a, int n, int x) {
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (a[mid] < x)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

constexpr int RHS_T = AccS::T;   // tile order of the multi-RHS products
enum { RT_ASM = 0, RT_DIAG = 1, RT_SYRK = 2, RT_OFF = 3, RHS_KINDS = 4 };

// Tasks of the multi-RHS products of one supernode with r RHS columns, n3
// DOF columns and b3 below rows (tiles of RHS_T): assemble (4 columns per
// task), L_ss^{-1} X (row tile x column tile), Z^T Z (lower column-tile
// pairs), L_21 Z (below-row tile x column tile).  The host evaluates the same
// counts at r = rmax for the list capacities.
__host__ __device__ inline void rhs_task_counts(int r, int n3, int b3, int c[RHS_KINDS]) {
  if (r <= 0) {
    c[RT_ASM] = c[RT_DIAG] = c[RT_SYRK] = c[RT_OFF] = 0;
    return;
  }
  const int tr = (r + RHS_T - 1) / RHS_T;
  c[RT_ASM] = (r + 3) / 4;
  c[RT_DIAG] = ((n3 + RHS_T - 1) / RHS_T) * tr;
  c[RT_SYRK] = tr * (tr + 1) / 2;
  c[RT_OFF] = ((b3 + RHS_T - 1) / RHS_T) * tr;
}

// k_rhs_plan (one block per height level): the contact range [lo, own, hi)
// of every supernode of the level (contacts are sorted by supernode; a range
// over the supernode's capacity, reachable only with duplicate ids, which are
// flagged, is emptied), then the level's task lists: one entry (supernode,
// tile row << 16 | tile column) per tile that has work, in supernode order,
// and the list lengths.  The products launch one workgroup per entry of the
// list's capacity; those past its length return after one uniform load (a
// grid laid out by supernode and static column capacity would have most of
// its workgroups find no columns, each after three dependent loads).
constexpr int PLAN_NT = 1024;     // threads
constexpr int PLAN_CHUNK = 256;   // supernodes per chunk (levels with more take several)
constexpr int PLAN_KEYS = 4096;
__global__ __launch_bounds__(PLAN_NT) void k_rhs_plan(int nc, const int *__restrict__ level_first,
                                                      const int *__restrict__ level_sup,
                                                      const SupDev *__restrict__ sup, const int *__restrict__ keys,
                                                      int *__restrict__ lohi, const int *__restrict__ task_off,
                                                      int *__restrict__ task_cnt, int2 *__restrict__ tasks) {
  __shared__ int pre[RHS_KINDS][PLAN_CHUNK];
  __shared__ int wsum[RHS_KINDS][PLAN_CHUNK / 64];
  __shared__ int wtot[RHS_KINDS];
  __shared__ int ssup[PLAN_CHUNK], sn3t[PLAN_CHUNK], sb3t[PLAN_CHUNK];
  __shared__ int skeys[PLAN_KEYS];
  const int l = blockIdx.x, tid = threadIdx.x, ln = tid & 63, wv = tid >> 6;
  const int first = level_first[l], last = level_first[l + 1];
  // the sorted keys are searched in LDS when they fit
  const int *kp = keys;
  if (nc <= PLAN_KEYS) {
    for (int i = tid; i < nc; i += PLAN_NT) skeys[i] = keys[i];
    __syncthreads();
    kp = skeys;
  }
  int run[RHS_KINDS] = {0, 0, 0, 0};
  for (int base = first; base < last; base += PLAN_CHUNK) {
    // ranges, task counts and their exclusive prefix over the chunk (waves
    // 0 .. PLAN_CHUNK / 64 - 1)
    const int q = base + tid;
    int c[RHS_KINDS] = {0, 0, 0, 0};
    if (tid < PLAN_CHUNK && q < last) {
      const int sn = level_sup[q];
      const SupDev &S = sup[sn];
      const int lo = lower_bound_i(kp, nc, S.first_desc);
      int own = lower_bound_i(kp, nc, sn);
      int hi = lower_bound_i(kp, nc, sn + 1);
      if (3 * (hi - lo) > S.rmax) own = hi = lo;
      lohi[3 * sn + 0] = lo;
      lohi[3 * sn + 1] = own;
      lohi[3 * sn + 2] = hi;
      const int n3 = 3 * S.ncol, b3 = 3 * S.nb;
      rhs_task_counts(3 * (hi - lo), n3, b3, c);
      ssup[tid] = sn;
      sn3t[tid] = (n3 + RHS_T - 1) / RHS_T;
      sb3t[tid] = (b3 + RHS_T - 1) / RHS_T;
    }
    int v[RHS_KINDS];
#pragma unroll
    for (int k = 0; k < RHS_KINDS; ++k) v[k] = c[k];
    if (tid < PLAN_CHUNK) {
      for (int o = 1; o < 64; o <<= 1) {
#pragma unroll
        for (int k = 0; k < RHS_KINDS; ++k) {
          const int t = __shfl_up(v[k], o, 64);
          if (ln >= o) v[k] += t;
        }
      }
      if (ln == 63) {
#pragma unroll
        for (int k = 0; k < RHS_KINDS; ++k) wsum[k][wv] = v[k];
      }
    }
    __syncthreads();
    if (tid < RHS_KINDS) {
      int acc = 0;
      for (int w = 0; w < PLAN_CHUNK / 64; ++w) {
        const int t = wsum[tid][w];
        wsum[tid][w] = acc;
        acc += t;
      }
      wtot[tid] = acc;
    }
    __syncthreads();
    if (tid < PLAN_CHUNK) {
#pragma unroll
      for (int k = 0; k < RHS_KINDS; ++k) pre[k][tid] = wsum[k][wv] + v[k] - c[k];
    }
    __syncthreads();
    // the chunk's tasks, all threads
    const int nq = min(PLAN_CHUNK, last - base);
    for (int k = 0; k < RHS_KINDS; ++k) {
      const int tot = wtot[k];
      int2 *out = tasks + task_off[RHS_KINDS * l + k] + run[k];
      for (int t = tid; t < tot; t += PLAN_NT) {
        int a = 0, b = nq;   // first q with pre > t; the task's supernode is the one before
        while (a < b) {
          const int mid = (a + b) >> 1;
          if (pre[k][mid] <= t)
            a = mid + 1;
          else
            b = mid;
        }
        const int qq = a - 1, u = t - pre[k][qq];
        int ti = u, tj = 0;
        if (k == RT_DIAG) {   // deepest row tiles first (their product runs over k < i0 + 64)
          ti = sn3t[qq] - 1 - u % sn3t[qq];
          tj = u / sn3t[qq];
        } else if (k == RT_SYRK) {
          tri_index(u, ti, tj);
        } else if (k == RT_OFF) {
          ti = u % sb3t[qq];
          tj = u / sb3t[qq];
        }
        out[t] = make_int2(ssup[qq], (ti << 16) | tj);
      }
      run[k] += tot;
    }
    __syncthreads();
  }
  if (tid < RHS_KINDS) task_cnt[RHS_KINDS * l + tid] = run[tid];
}

// ---- multi-RHS forward ------------------------------------------------------

// X_s column by column (one wave per column, 4 columns per task): a column
// of an own contact is a unit vector of H^T (or a column of J^T = H^T C^T
// when frames are given); a column of a contact below a child is the child's
// below-row part extended into the front rows (extend-add through invmap).
// With a residual R (the correction solve of the refinement), the columns
// carry R_s on the supernode's own rows instead of the unit vectors, plus
// the children's parts.  Everything that identifies the column is uniform
// over the wave.
template <class E>
__device__ inline void rhs_assemble_column(const SupDev *__restrict__ sup, int s, int jc, int l,
                                           const int *__restrict__ child, const int *__restrict__ invmap_off,
                                           const int *__restrict__ invmap, const int *__restrict__ lohi,
                                           const int *__restrict__ order, const int *__restrict__ node_ids,
                                           const int *__restrict__ iperm, const double *__restrict__ frames,
                                           const double *__restrict__ R, E *__restrict__ X) {
  const SupDev S = sup[s];
  const int lo = lohi[3 * s], own = lohi[3 * s + 1], hi = lohi[3 * s + 2];
  const int r = 3 * (hi - lo);
  if (jc >= r) return;
  const int n3 = 3 * S.ncol, f = 3 * (S.ncol + S.nb);
  E *Xc = X + S.x_off + (long)jc * f;
  const double *Rc = R ? R + S.z_off + (long)jc * n3 : nullptr;
  const int p = lo + jc / 3, a = jc % 3;
  if (p >= own) {
    if (Rc) {
      for (int i = l; i < f; i += 64) Xc[i] = (i < n3) ? E(Rc[i]) : E(0);
      return;
    }
    const int c = order[p];
    const int base = 3 * (iperm[node_ids[c]] - S.col0);
    for (int i = l; i < f; i += 64) {
      double v;
      if (frames == nullptr)
        v = (i == base + a) ? 1.0 : 0.0;
      else
        v = (i >= base && i < base + 3) ? frames[9L * c + 3 * a + (i - base)] : 0.0;
      Xc[i] = E(v);
    }
    return;
  }
  int cc = -1, clo = 0;
  for (int q = 0; q < S.nchild; ++q) {
    const int ch = child[S.child_off + q];
    if (p >= lohi[3 * ch] && p < lohi[3 * ch + 2]) {
      cc = q;
      clo = lohi[3 * ch];
      break;
    }
  }
  if (cc < 0) {   // not below any child (cannot happen for sorted contacts)
    for (int i = l; i < f; i += 64) Xc[i] = E(0);
    return;
  }
  const SupDev C = sup[child[S.child_off + cc]];
  const int fc = 3 * (C.ncol + C.nb);
  const int *im = invmap + invmap_off[S.child_off + cc];
  const E *src = X + C.x_off + (long)(jc - 3 * (clo - lo)) * fc + 3 * C.ncol;
  for (int i = l; i < f; i += 64) {
    const int ii = im[i / 3];
    E v = (ii >= 0) ? src[3 * ii + i % 3] : E(0);
    if (Rc && i < n3) v += E(Rc[i]);
    Xc[i] = v;
  }
}

// The product kernels take task blockIdx.x of their level's list; the grid is
// the list's capacity and the workgroups past its length return after one
// uniform load.
template <class E>
__global__ __launch_bounds__(256) void k_rhs_assemble(const SupDev *__restrict__ sup, const int2 *__restrict__ tasks,
                                                      const int *__restrict__ ntask, const int *__restrict__ child,
                                                      const int *__restrict__ invmap_off,
                                                      const int *__restrict__ invmap, const int *__restrict__ lohi,
                                                      const int *__restrict__ order, const int *__restrict__ node_ids,
                                                      const int *__restrict__ iperm, const double *__restrict__ frames,
                                                      const double *__restrict__ R, E *__restrict__ X) {
  if ((int)blockIdx.x >= *ntask) return;
  const int2 tk = tasks[blockIdx.x];
  rhs_assemble_column<E>(sup, tk.x, 4 * (tk.y >> 16) + (threadIdx.x >> 6), threadIdx.x & 63, child, invmap_off,
                         invmap, lohi, order, node_ids, iperm, frames, R, X);
}

// Z_s = L_ss^{-1} X_s[:n_s], one 64x64 tile per task.  z64 (FP32 solves of
// the mixed-precision build): 1 also stores the tile into the FP64 Z,
// 2 adds it there (a refinement correction).
template <class Ac>
__global__ __launch_bounds__(256) void k_rhs_diag(const SupDev *__restrict__ sup, const int2 *__restrict__ tasks,
                                                  const int *__restrict__ ntask, const int *__restrict__ lohi,
                                                  const typename Ac::elem *__restrict__ linv,
                                                  const typename Ac::elem *__restrict__ X,
                                                  typename Ac::elem *__restrict__ Z, double *__restrict__ Z64,
                                                  int z64) {
  typedef typename Ac::elem E;
  constexpr int T = Ac::T;
  __shared__ E lds[Ac::LDS];
  if ((int)blockIdx.x >= *ntask) return;
  const int2 tk = tasks[blockIdx.x];
  const int s = tk.x;
  const SupDev S = sup[s];
  const int r = 3 * (lohi[3 * s + 2] - lohi[3 * s]);
  const int n3 = 3 * S.ncol, f = 3 * (S.ncol + S.nb);
  const int i0 = T * (tk.y >> 16), j0 = T * (tk.y & 0xffff);
  if (i0 >= n3 || j0 >= r) return;
  const int M = min(T, n3 - i0), N = min(T, r - j0);
  const int kend = min(n3, i0 + T);
  Ac acc;
  acc.zero();
  acc.template acc<true, false>(linv + S.linv_off + i0, 1, n3, X + S.x_off + (long)j0 * f, 1, f, M, N, 0, kend,
                                lds);
  E *Zs = Z + S.z_off;
  double *Z64s = Z64 ? Z64 + S.z_off : nullptr;
  acc.for_each([&](int i, int j, E v) {
    if (i < M && j < N) {
      const long e = (long)(i0 + i) + (long)(j0 + j) * n3;
      Zs[e] = v;
      if (z64 == 1) Z64s[e] = (double)v;
      if (z64 == 2) Z64s[e] += (double)v;
    }
  });
}

// X_s[n_s:] -= L_21 Z_s, one tile per task
template <class Ac>
__global__ __launch_bounds__(256) void k_rhs_off(const SupDev *__restrict__ sup, const int2 *__restrict__ tasks,
                                                 const int *__restrict__ ntask, const int *__restrict__ lohi,
                                                 const typename Ac::elem *__restrict__ front,
                                                 const typename Ac::elem *__restrict__ Z,
                                                 typename Ac::elem *__restrict__ X) {
  typedef typename Ac::elem E;
  constexpr int T = Ac::T;
  __shared__ E lds[Ac::LDS];
  if ((int)blockIdx.x >= *ntask) return;
  const int2 tk = tasks[blockIdx.x];
  const int s = tk.x;
  const SupDev S = sup[s];
  const int r = 3 * (lohi[3 * s + 2] - lohi[3 * s]);
  const int n3 = 3 * S.ncol, b3 = 3 * S.nb, f = n3 + b3;
  const int i0 = T * (tk.y >> 16), j0 = T * (tk.y & 0xffff);
  if (i0 >= b3 || j0 >= r) return;
  const int M = min(T, b3 - i0), N = min(T, r - j0);
  Ac acc;
  acc.zero();
  acc.template acc<true, false>(front + S.front_off + n3 + i0, 1, f, Z + S.z_off + (long)j0 * n3, 1, n3, M, N, 0,
                                n3, lds);
  E *Xs = X + S.x_off;
  acc.for_each([&](int i, int j, E v) {
    if (i < M && j < N) Xs[(long)(n3 + i0 + i) + (long)(j0 + j) * f] -= v;
  });
}

// Residual of the forward solve on a supernode's own rows (FP64, the
// refinement of the mixed-precision build): R_s = X_s[:n_s] - L_ss Z_s with
// X_s assembled in FP64 from the unit columns and the children's FP64
// updates; L_ss is the lower triangle of the front's diagonal block.
template <class Ac>
__global__ __launch_bounds__(256) void k_rhs_resid(const SupDev *__restrict__ sup, const int2 *__restrict__ tasks,
                                                   const int *__restrict__ ntask, const int *__restrict__ lohi,
                                                   const double *__restrict__ front, const double *__restrict__ X,
                                                   const double *__restrict__ Z, double *__restrict__ R) {
  constexpr int T = Ac::T;
  __shared__ double lds[Ac::LDS];
  if ((int)blockIdx.x >= *ntask) return;
  const int2 tk = tasks[blockIdx.x];
  const int s = tk.x;
  const SupDev S = sup[s];
  const int r = 3 * (lohi[3 * s + 2] - lohi[3 * s]);
  const int n3 = 3 * S.ncol, f = 3 * (S.ncol + S.nb);
  const int i0 = T * (tk.y >> 16), j0 = T * (tk.y & 0xffff);
  if (i0 >= n3 || j0 >= r) return;
  const int M = min(T, n3 - i0), N = min(T, r - j0);
  const int kend = min(n3, i0 + T);
  Ac acc;
  acc.zero();
  // A(i, k) = L_ss(i0 + i, k), zero above the diagonal (k > i0 + i)
  acc.template acc<true, false, true>(front + S.front_off + i0, 1, f, Z + S.z_off + (long)j0 * n3, 1, n3, M, N, 0,
                                      kend, lds, i0);
  const double *Xs = X + S.x_off;
  double *Rs = R + S.z_off;
  acc.for_each([&](int i, int j, double v) {
    if (i < M && j < N) Rs[(long)(i0 + i) + (long)(j0 + j) * n3] = Xs[(long)(i0 + i) + (long)(j0 + j) * f] - v;
  });
}

// Wp[3lo + i][3lo + j] += sum_k Z(k, i) Z(k, j), one lower tile of the r x r
// block per task
template <class Ac>
__global__ __launch_bounds__(256) void k_rhs_syrk(const SupDev *__restrict__ sup, const int2 *__restrict__ tasks,
                                                  const int *__restrict__ ntask, const int *__restrict__ lohi,
                                                  const double *__restrict__ Z, int m, double *__restrict__ Wp) {
  constexpr int T = Ac::T;
  __shared__ double lds[Ac::LDS];
  if ((int)blockIdx.x >= *ntask) return;
  const int2 tk = tasks[blockIdx.x];
  const int s = tk.x;
  const SupDev S = sup[s];
  const int lo = lohi[3 * s];
  const int r = 3 * (lohi[3 * s + 2] - lo);
  const int i0 = T * (tk.y >> 16), j0 = T * (tk.y & 0xffff);
  if (i0 >= r || j0 > i0) return;
  const int n3 = 3 * S.ncol;
  const int M = min(T, r - i0), N = min(T, r - j0);
  const double *Zs = Z + S.z_off;
  Ac acc;
  acc.zero();
  acc.template acc<false, false>(Zs + (long)i0 * n3, n3, 1, Zs + (long)j0 * n3, 1, n3, M, N, 0, n3, lds);
  const long base = (long)(3 * lo) * m + 3 * lo;
  acc.for_each([&](int i, int j, double v) {
    if (i < M && j < N) Wp[base + (long)(i0 + i) * m + (j0 + j)] += v;
  });
}

__global__ void k_fill(long n, double v, double *__restrict__ x) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) x[i] = v;
}

// Mirror the lower triangle of Wp (supernode order) into the upper one,
// 64 x 64 tiles through LDS so that both the read and the transposed write
// are coalesced; tiles (I >= J) of the lower triangle.
__global__ __launch_bounds__(256) void k_wp_mirror(int m, double *__restrict__ Wp) {
  __shared__ double t[64][65];
  const int nt = (m + 63) / 64;
  if ((int)blockIdx.x >= nt * (nt + 1) / 2) return;
  int I, J;
  tri_index(blockIdx.x, I, J);
  const int i0 = 64 * I, j0 = 64 * J;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int r = ty; r < 64; r += 4) {
    const int i = i0 + r, j = j0 + tx;
    t[r][tx] = (i < m && j < m) ? Wp[(long)i * m + j] : 0.0;
  }
  __syncthreads();
  // upper entry (j0 + r, i0 + tx) = lower entry (i0 + tx, j0 + r) when strictly below the diagonal
  for (int r = ty; r < 64; r += 4) {
    const int row = j0 + r, col = i0 + tx;
    if (row < m && col < m && col > row) Wp[(long)row * m + col] = t[tx][r];
  }
}

// W_H[3c+a][3c'+b] = Wp[3 pos(c) + a][3 pos(c') + b] (Wp symmetric): one
// block per output row, the source row stays in cache.
template <class TW>
__global__ __launch_bounds__(256) void k_wh_unpermute(int nc, const int *__restrict__ pos, const double *__restrict__ Wp,
                                                      TW *__restrict__ WH) {
  const int m = 3 * nc;
  const int i = blockIdx.x;
  const double *src = Wp + (long)(3 * pos[i / 3] + i % 3) * m;
  TW *dst = WH + (long)i * m;
  for (int j = threadIdx.x; j < m; j += 256) dst[j] = (TW)src[3 * pos[j / 3] + j % 3];
}

__global__ void k_to_float(long n, const double *__restrict__ x, float *__restrict__ y) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    y[i] = (float)x[i];
}

__global__ void k_to_double(long n, const float *__restrict__ x, double *__restrict__ y) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    y[i] = (double)x[i];
}

// Mapped contacts (Eq. 6): contact a is the point sum_k w_ak x(u_ak) over up
// to four slots (unused slots: index -1), so H = Hw Hn with Hn the nodal
// selection of the distinct nodes and
//   W_H[3a+i][3b+j] = sum_{k,l} w_ak w_bl W_N[3 u_ak + i][3 u_bl + j],
// W_N = Hn A^-1 Hn^T (built by the nodal path).  One block per contact row
// a, threads over b.  The sixteen terms are summed in an order that is the
// same for (a, b) and (b, a) -- diagonal slot pairs, then each off-diagonal
// pair (k, l) as t_kl + t_lk -- with products and sums rounded separately
// (no contraction), so W_H is exactly symmetric like W_N.
__global__ __launch_bounds__(256) void k_wh_expand(int nc, int nu3, const int *__restrict__ idx,
                                                   const double *__restrict__ wts, const double *__restrict__ WN,
                                                   double *__restrict__ WH) {
  const int a = blockIdx.x;
  int ua[4];
  double wa[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    ua[k] = idx[4 * a + k];
    wa[k] = ua[k] >= 0 ? wts[4 * a + k] : 0.0;
  }
  const long m = 3L * nc;
  for (int b = threadIdx.x; b < nc; b += blockDim.x) {
    int ub[4];
    double wb[4];
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      ub[l] = idx[4 * b + l];
      wb[l] = ub[l] >= 0 ? wts[4 * b + l] : 0.0;
    }
    // t(k, l)[i][j] = (w_ak w_bl) W_N[3 u_ak + i][3 u_bl + j], 0 for an unused slot
    auto term = [&](int k, int l, int i, int j) -> double {
      if (ua[k] < 0 || ub[l] < 0) return 0.0;
      return __dmul_rn(__dmul_rn(wa[k], wb[l]), WN[(long)(3 * ua[k] + i) * nu3 + 3 * ub[l] + j]);
    };
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        double acc = term(0, 0, i, j);
#pragma unroll
        for (int k = 1; k < 4; ++k) acc = __dadd_rn(acc, term(k, k, i, j));
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
          for (int l = k + 1; l < 4; ++l) acc = __dadd_rn(acc, __dadd_rn(term(k, l, i, j), term(l, k, i, j)));
        WH[(3L * a + i) * m + 3L * b + j] = acc;
      }
    }
  }
}

// ---- single RHS -------------------------------------------------------------

// Single-RHS products, 1024 threads per block.  Column-major A times x: lane
// = row (64 rows, coalesced), wave = k-phase (16 phases), four independent
// accumulators per thread, phases summed in a fixed order through LDS.
// Transposed products: one wave per column, 16 columns per block, the
// vector staged in LDS once per block.
constexpr int GV_R = 64, GV_P = 16, GV_X = 4096;
constexpr int ZF_K = 256;   // columns of Z per chunk of the Z f product

__device__ inline double gemv_part(const double *__restrict__ A, long lda, const double *__restrict__ x, int i,
                                   int nrows, int k0, int k1, int ph) {
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  if (i < nrows) {
    int k = k0 + ph;
    for (; k + 3 * GV_P < k1; k += 4 * GV_P) {
      a0 = fma(A[i + (long)k * lda], x[k], a0);
      a1 = fma(A[i + (long)(k + GV_P) * lda], x[k + GV_P], a1);
      a2 = fma(A[i + (long)(k + 2 * GV_P) * lda], x[k + 2 * GV_P], a2);
      a3 = fma(A[i + (long)(k + 3 * GV_P) * lda], x[k + 3 * GV_P], a3);
    }
    for (; k < k1; k += GV_P) a0 = fma(A[i + (long)k * lda], x[k], a0);
  }
  return (a0 + a1) + (a2 + a3);
}

// Sum of the 16 phase partials of row r (valid in wave 0).
__device__ inline double phase_sum(double v, double (*part)[GV_R + 1]) {
  const int r = threadIdx.x & 63, ph = threadIdx.x >> 6;
  part[ph][r] = v;
  __syncthreads();
  double t = 0.0;
  if (ph == 0)
    for (int q = 0; q < GV_P; ++q) t += part[q][r];
  return t;
}

// Entry i of the single-RHS front of supernode S (Eq. 12 forward half): the
// permuted right-hand side on its own columns plus the children's update
// entries mapped onto row i (extend-add), children in order.
__device__ inline double fwd1_front(const SupDev &S, int i, const SupDev *__restrict__ sup,
                                    const int *__restrict__ child, const int *__restrict__ invmap_off,
                                    const int *__restrict__ invmap, const int *__restrict__ perm,
                                    const double *__restrict__ b, const double *__restrict__ x1) {
  const int n3 = 3 * S.ncol;
  double v = (i < n3) ? b[3 * perm[S.col0 + i / 3] + i % 3] : 0.0;
  for (int c = 0; c < S.nchild; ++c) {
    const int ii = invmap[invmap_off[S.child_off + c] + i / 3];
    if (ii >= 0) {
      const SupDev C = sup[child[S.child_off + c]];
      v += x1[C.x1_off + 3 * C.ncol + 3 * ii + i % 3];
    }
  }
  return v;
}

// The single-RHS products take block x from a static task list of their
// level: (supernode of the level, block of 64 rows or 16 columns), only the
// blocks a supernode has.  Split-K (top tree levels, where a level has too
// few row blocks to fill the GPU): block y = chunk of k; each block writes
// the sums over its chunk to part[(task * nsplit + chunk) * 64 + row] and
// k_fwd1_fin adds the nsplit partials in chunk order.  nsplit = 1: the row
// block's sums are final.  Returns true when they are (wave 0: row sums).
__device__ inline bool fwd1_split_store(double t, double *__restrict__ part) {
  const int nsplit = gridDim.y;
  if (nsplit == 1) return true;
  const int r = threadIdx.x & 63, ph = threadIdx.x >> 6;
  if (ph == 0) part[((long)blockIdx.x * nsplit + blockIdx.y) * GV_R + r] = t;
  return false;
}

// Chunk [ka, kb) of k in [0, kend) for chunk ks of nsplit (multiples of GV_P).
__device__ inline void fwd1_chunk(int kend, int nsplit, int ks, int &ka, int &kb) {
  const int kc = ((kend + nsplit - 1) / nsplit + GV_P - 1) / GV_P * GV_P;
  ka = min(kend, ks * kc);
  kb = min(kend, ka + kc);
}

// y[3 col0 + i] = sum_{k <= i} Linv(i, k) x1_s[k]; the front entries it needs
// are assembled on the fly into LDS (GV_X at a time)
__global__ __launch_bounds__(1024) void k_fwd1_diag(const SupDev *__restrict__ sup, const int *__restrict__ level_sup,
                                                    const int2 *__restrict__ tasks, const int *__restrict__ child,
                                                    const int *__restrict__ invmap_off, const int *__restrict__ invmap,
                                                    const int *__restrict__ perm, const double *__restrict__ b,
                                                    const double *__restrict__ linv, const double *__restrict__ x1,
                                                    double *__restrict__ y, double *__restrict__ part) {
  __shared__ double ps[GV_P][GV_R + 1];
  __shared__ double xs[GV_X];
  const int2 tk = tasks[blockIdx.x];
  const SupDev S = sup[level_sup[tk.x]];
  const int n3 = 3 * S.ncol;
  const int i0 = GV_R * tk.y;
  const int r = threadIdx.x & 63, ph = threadIdx.x >> 6, i = i0 + r;
  const int kend = min(n3, i0 + GV_R);
  int ka, kb;
  fwd1_chunk(kend, gridDim.y, blockIdx.y, ka, kb);
  double v = 0.0;
  for (int kk = ka; kk < kb; kk += GV_X) {
    const int kn = min(kb, kk + GV_X);
    __syncthreads();
    for (int k = kk + threadIdx.x; k < kn; k += 1024)
      xs[k - kk] = fwd1_front(S, k, sup, child, invmap_off, invmap, perm, b, x1);
    __syncthreads();
    v += gemv_part(linv + S.linv_off, n3, xs - kk, i, n3, kk, kn, ph);
  }
  const double t = phase_sum(v, ps);
  if (!fwd1_split_store(t, part)) return;
  if (ph == 0 && i < n3) y[3 * S.col0 + i] = t;
}

// x1_s[n_s + i] = front(n_s + i) - sum_k L21(i, k) y_s[k]
__global__ __launch_bounds__(1024) void k_fwd1_off(const SupDev *__restrict__ sup, const int *__restrict__ level_sup,
                                                   const int2 *__restrict__ tasks, const int *__restrict__ child,
                                                   const int *__restrict__ invmap_off,
                                                   const int *__restrict__ invmap, const int *__restrict__ perm,
                                                   const double *__restrict__ b, const double *__restrict__ front,
                                                   const double *__restrict__ y, double *__restrict__ x1,
                                                   double *__restrict__ part) {
  __shared__ double ps[GV_P][GV_R + 1];
  const int2 tk = tasks[blockIdx.x];
  const SupDev S = sup[level_sup[tk.x]];
  const int n3 = 3 * S.ncol, b3 = 3 * S.nb, f = n3 + b3;
  const int i0 = GV_R * tk.y;
  const int r = threadIdx.x & 63, ph = threadIdx.x >> 6, i = i0 + r;
  int ka, kb;
  fwd1_chunk(n3, gridDim.y, blockIdx.y, ka, kb);
  const double v = gemv_part(front + S.front_off + n3, f, y + 3 * S.col0, i, b3, ka, kb, ph);
  const double t = phase_sum(v, ps);
  if (!fwd1_split_store(t, part)) return;
  if (ph == 0 && i < b3)
    x1[S.x1_off + n3 + i] = fwd1_front(S, n3 + i, sup, child, invmap_off, invmap, perm, b, x1) - t;
}

// The sums of split products (one wave per row block): off = 0 writes y of
// the diagonal product, off = 1 the below rows of x1.
__global__ __launch_bounds__(64) void k_fwd1_fin(const SupDev *__restrict__ sup, const int *__restrict__ level_sup,
                                                 const int2 *__restrict__ tasks, const int *__restrict__ child,
                                                 const int *__restrict__ invmap_off,
                                                 const int *__restrict__ invmap, const int *__restrict__ perm,
                                                 const double *__restrict__ b, int off, int nsplit,
                                                 const double *__restrict__ part, double *__restrict__ y,
                                                 double *__restrict__ x1) {
  const int2 tk = tasks[blockIdx.x];
  const SupDev S = sup[level_sup[tk.x]];
  const int n3 = 3 * S.ncol, rows = off ? 3 * S.nb : n3;
  const int i = GV_R * tk.y + (int)threadIdx.x;
  if (i >= rows) return;
  double t = 0.0;
  for (int q = 0; q < nsplit; ++q) t += part[((long)blockIdx.x * nsplit + q) * GV_R + threadIdx.x];
  if (off)
    x1[S.x1_off + n3 + i] = fwd1_front(S, n3 + i, sup, child, invmap_off, invmap, perm, b, x1) - t;
  else
    y[3 * S.col0 + i] = t;
}

// y_s[j] -= sum_i L21(i, j) x[below row i]
__global__ __launch_bounds__(1024) void k_bwd1_off(const SupDev *__restrict__ sup, const int *__restrict__ level_sup,
                                                   const int2 *__restrict__ tasks, const int *__restrict__ rows,
                                                   const double *__restrict__ front, const double *__restrict__ xp,
                                                   double *__restrict__ y) {
  __shared__ double xg[GV_X];
  const int2 tk = tasks[blockIdx.x];
  const SupDev S = sup[level_sup[tk.x]];
  const int n3 = 3 * S.ncol, b3 = 3 * S.nb, f = n3 + b3;
  const int j0 = GV_P * tk.y;
  const int *rw = rows + S.rows_off;
  const int bs = min(b3, GV_X);
  for (int i = threadIdx.x; i < bs; i += 1024) xg[i] = xp[3 * rw[i / 3] + i % 3];
  __syncthreads();
  const int j = j0 + (threadIdx.x >> 6), l = threadIdx.x & 63;
  if (j >= n3) return;
  const double *F = front + S.front_off + n3 + (long)j * f;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int i = l;
  for (; i + 192 < bs; i += 256) {
    a0 = fma(F[i], xg[i], a0);
    a1 = fma(F[i + 64], xg[i + 64], a1);
    a2 = fma(F[i + 128], xg[i + 128], a2);
    a3 = fma(F[i + 192], xg[i + 192], a3);
  }
  for (; i < bs; i += 64) a0 = fma(F[i], xg[i], a0);
  for (; i < b3; i += 64) a0 = fma(F[i], xp[3 * rw[i / 3] + i % 3], a0);
  double acc = (a0 + a1) + (a2 + a3);
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (l == 0) y[3 * S.col0 + j] -= acc;
}

// xp[3 col0 + j] = sum_{i >= j} Linv(i, j) y_s[i]
__global__ __launch_bounds__(1024) void k_bwd1_diag(const SupDev *__restrict__ sup, const int *__restrict__ level_sup,
                                                    const int2 *__restrict__ tasks, const double *__restrict__ linv,
                                                    const double *__restrict__ y, double *__restrict__ xp) {
  __shared__ double yg[GV_X];
  const int2 tk = tasks[blockIdx.x];
  const SupDev S = sup[level_sup[tk.x]];
  const int n3 = 3 * S.ncol;
  const int j0 = GV_P * tk.y;
  const double *ys = y + 3 * S.col0;
  const int ns = min(n3, GV_X);
  for (int i = j0 + threadIdx.x; i < ns; i += 1024) yg[i] = ys[i];
  __syncthreads();
  const int j = j0 + (threadIdx.x >> 6), l = threadIdx.x & 63;
  if (j >= n3) return;
  const double *Lc = linv + S.linv_off + (long)j * n3;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int i = j + l;
  for (; i + 192 < ns; i += 256) {
    a0 = fma(Lc[i], yg[i], a0);
    a1 = fma(Lc[i + 64], yg[i + 64], a1);
    a2 = fma(Lc[i + 128], yg[i + 128], a2);
    a3 = fma(Lc[i + 192], yg[i + 192], a3);
  }
  for (; i < ns; i += 64) a0 = fma(Lc[i], yg[i], a0);
  for (; i < n3; i += 64) a0 = fma(Lc[i], ys[i], a0);
  double acc = (a0 + a1) + (a2 + a3);
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (l == 0) xp[3 * S.col0 + j] = acc;
}

__global__ void k_unpermute_vec(int N, const int *__restrict__ perm, const double *__restrict__ xp,
                                double *__restrict__ x) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  int v = perm[p];
  x[3 * v] = xp[3 * p];
  x[3 * v + 1] = xp[3 * p + 1];
  x[3 * v + 2] = xp[3 * p + 2];
}

}  // namespace

namespace {

void backward_solve(icr_scene *s, double *x) {
  auto &F = s->fac;
  hipStream_t st = s->stream;
  const int nl = (int)F.levels.size();
  double *y = F.d_y, *xp = F.d_y + s->mesh.n;
  for (int l = nl - 1; l >= 0; --l) {
    const LevelInfo &L = F.levels[l];
    if (!L.count) continue;
    const int *ls = F.d_level_sup + L.first;
    const int2 *tb = F.d_srhs_tasks + L.srhs_off[SR_BWD];
    const unsigned nb = (unsigned)L.srhs_cnt[SR_BWD];
    if (L.max_b3 > 0) {
      k_bwd1_off<<<nb, 1024, 0, st>>>(F.d_sup, ls, tb, F.d_rows, F.d_front, xp, y);
      ICR_LAUNCH_CHECK();
    }
    k_bwd1_diag<<<nb, 1024, 0, st>>>(F.d_sup, ls, tb, F.d_linv, y, xp);
    ICR_LAUNCH_CHECK();
  }
  k_unpermute_vec<<<cdiv(s->mesh.N, 256), 256, 0, st>>>(s->mesh.N, F.d_perm, xp, x);
  ICR_LAUNCH_CHECK();
}

// y[3 col0_s + i] = sum_c Z_s(i, c) f[contact at column c]: the forward half of
// A^-1 H^T f reuses Z = L^-1 P H^T from the W_H build of the same contacts.
// k_zf_part: one task = 64 rows x one chunk of ZF_K columns of Z_s, partial
// sums to part[off + chunk n3 + row]; k_zf_sum adds the chunks in order.
__global__ __launch_bounds__(1024) void k_zf_part(const int4 *__restrict__ tasks, const SupDev *__restrict__ sup,
                                                  const int *__restrict__ lohi, const double *__restrict__ Z,
                                                  const double *__restrict__ fpos, double *__restrict__ part) {
  __shared__ double ps[GV_P][GV_R + 1];
  const int4 tk = tasks[blockIdx.x];
  const int s = tk.x, i0 = tk.y, k0 = tk.z;
  const SupDev S = sup[s];
  const int n3 = 3 * S.ncol;
  const int lo = lohi[3 * s], r = 3 * (lohi[3 * s + 2] - lo);
  if (k0 >= r && k0 > 0) return;   // chunk beyond this call's columns (chunk 0 always writes)
  const int rr = threadIdx.x & 63, ph = threadIdx.x >> 6, i = i0 + rr;
  const double v = gemv_part(Z + S.z_off, n3, fpos + 3 * lo, i, n3, k0, min(r, k0 + ZF_K), ph);
  const double t = phase_sum(v, ps);
  if (ph == 0 && i < n3) part[tk.w + (long)(k0 / ZF_K) * n3 + i] = t;
}
__global__ void k_zf_sum(const int4 *__restrict__ tasks, const SupDev *__restrict__ sup,
                         const int *__restrict__ lohi, const double *__restrict__ part, double *__restrict__ y) {
  const int4 tk = tasks[blockIdx.x];
  const int s = tk.x, i = tk.y + (int)threadIdx.x;
  const SupDev S = sup[s];
  const int n3 = 3 * S.ncol;
  if (i >= n3) return;
  const int r = 3 * (lohi[3 * s + 2] - lohi[3 * s]);
  const int nch = max(1, (r + ZF_K - 1) / ZF_K);
  double acc = 0.0;
  for (int ch = 0; ch < nch; ++ch) acc += part[tk.w + (long)ch * n3 + i];
  y[3 * S.col0 + i] = acc;
}

// fpos[3 p + a] = f[3 order[p] + a]
__global__ void k_gather_fpos(int nc, const int *__restrict__ order, const double *__restrict__ f,
                              double *__restrict__ fpos) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 3 * nc) return;
  fpos[e] = f[3 * order[e / 3] + e % 3];
}

}  // namespace

void single_rhs_solve(icr_scene *s, const double *b, double *x) {
  auto &F = s->fac;
  hipStream_t st = s->stream;
  const int nl = (int)F.levels.size();
  double *y = F.d_y;
  for (int l = 0; l < nl; ++l) {
    const LevelInfo &L = F.levels[l];
    if (!L.count) continue;
    const int *ls = F.d_level_sup + L.first;
    const int2 *td = F.d_srhs_tasks + L.srhs_off[SR_FWD_DIAG], *to = F.d_srhs_tasks + L.srhs_off[SR_FWD_OFF];
    const unsigned nd = (unsigned)L.srhs_cnt[SR_FWD_DIAG], no = (unsigned)L.srhs_cnt[SR_FWD_OFF];
    k_fwd1_diag<<<dim3(nd, L.fwd_split_diag), 1024, 0, st>>>(F.d_sup, ls, td, F.d_child, F.d_invmap_off, F.d_invmap,
                                                              F.d_perm, b, F.d_linv, F.d_x1, y, F.d_fwd_part);
    ICR_LAUNCH_CHECK();
    if (L.fwd_split_diag > 1) {
      k_fwd1_fin<<<nd, 64, 0, st>>>(F.d_sup, ls, td, F.d_child, F.d_invmap_off, F.d_invmap, F.d_perm, b, 0,
                                    L.fwd_split_diag, F.d_fwd_part, y, F.d_x1);
      ICR_LAUNCH_CHECK();
    }
    if (no > 0) {
      k_fwd1_off<<<dim3(no, L.fwd_split_off), 1024, 0, st>>>(F.d_sup, ls, to, F.d_child, F.d_invmap_off, F.d_invmap,
                                                              F.d_perm, b, F.d_front, y, F.d_x1, F.d_fwd_part);
      ICR_LAUNCH_CHECK();
      if (L.fwd_split_off > 1) {
        k_fwd1_fin<<<no, 64, 0, st>>>(F.d_sup, ls, to, F.d_child, F.d_invmap_off, F.d_invmap, F.d_perm, b, 1,
                                      L.fwd_split_off, F.d_fwd_part, y, F.d_x1);
        ICR_LAUNCH_CHECK();
      }
    }
  }
  backward_solve(s, x);
}

void contact_force_solve(icr_scene *s, const double *f, double *x) {
  auto &F = s->fac;
  const int nc = s->last_build_nc;
  k_gather_fpos<<<cdiv(3 * nc, 256), 256, 0, s->stream>>>(nc, F.d_order, f, F.d_fpos);
  ICR_LAUNCH_CHECK();
  k_zf_part<<<F.n_zf_tasks, 1024, 0, s->stream>>>(F.d_zf_tasks, F.d_sup, F.d_lohi, F.d_Z, F.d_fpos, F.d_zf_part);
  ICR_LAUNCH_CHECK();
  k_zf_sum<<<F.n_zf_sum_tasks, GV_R, 0, s->stream>>>(F.d_zf_tasks, F.d_sup, F.d_lohi, F.d_zf_part, F.d_y);
  ICR_LAUNCH_CHECK();
  backward_solve(s, x);
}

void launch_wh_expand(hipStream_t st, int nc, int nu, const int *idx, const double *w, const double *WN, double *WH) {
  k_wh_expand<<<nc, 256, 0, st>>>(nc, 3 * nu, idx, w, WN, WH);
  ICR_LAUNCH_CHECK();
}

void launch_narrow(icr_scene *s, const double *x, float *y, long n) {
  k_to_float<<<(unsigned)std::min<long>(1024, (n + 255) / 256), 256, 0, s->stream>>>(n, x, y);
  ICR_LAUNCH_CHECK();
}

void launch_widen(icr_scene *s, const float *x, double *y, long n) {
  k_to_double<<<(unsigned)std::min<long>(1024, (n + 255) / 256), 256, 0, s->stream>>>(n, x, y);
  ICR_LAUNCH_CHECK();
}

void launch_fill(icr_scene *s, double *x, long n, double v) {
  k_fill<<<(unsigned)std::min<long>(1024, (n + 255) / 256), 256, 0, s->stream>>>(n, v, x);
  ICR_LAUNCH_CHECK();
}

void ensure_rhs_capacity(icr_scene *s, int nc) {
  if (s->overlap && !s->side) {
    ICR_HIP(hipStreamCreateWithFlags(&s->side, hipStreamNonBlocking));
    ICR_HIP(hipEventCreateWithFlags(&s->ev_fork, hipEventDisableTiming));
    ICR_HIP(hipEventCreateWithFlags(&s->ev_join, hipEventDisableTiming));
  }
  auto &F = s->fac;
  if (nc <= F.nc_cap) return;
  s->epoch++;
  ICR_HIP(hipStreamSynchronize(s->stream));
  F.rhs_arena.release();
  long long xo = 0, zo = 0;
  for (int i = 0; i < (int)F.sup.size(); ++i) {
    SupDev &d = F.sup[i];
    int rmax = 3 * std::min(nc, d.region_nodes);
    d.rmax = rmax;
    d.x_off = xo;
    d.z_off = zo;
    xo += (long long)3 * (d.ncol + d.nb) * rmax;
    zo += (long long)3 * d.ncol * rmax;
  }
  F.d_X = F.rhs_arena.alloc<double>(xo);
  F.d_Z = F.rhs_arena.alloc<double>(zo);
  F.x_elems = xo;
  F.z_elems = zo;
  F.mixed_arena.release();   // sized for the previous offsets
  F.mixed_cap = 0;
  {
    // task-list capacities per (level, kind): the counts at r = rmax
    const int nlev = (int)F.levels.size();
    F.rhs_cap.assign(RHS_KINDS * nlev, 0);
    F.rhs_off.assign(RHS_KINDS * nlev, 0);
    std::vector<int> level_first(nlev + 1, 0);
    long long tot = 0;
    for (int l = 0; l < nlev; ++l) {
      const LevelInfo &L = F.levels[l];
      level_first[l] = L.first;
      level_first[l + 1] = L.first + L.count;
      for (int q = 0; q < L.count; ++q) {
        const SupDev &d = F.sup[F.sym.level_sup[L.first + q]];
        int c[RHS_KINDS];
        rhs_task_counts(d.rmax, 3 * d.ncol, 3 * d.nb, c);
        for (int k = 0; k < RHS_KINDS; ++k) F.rhs_cap[RHS_KINDS * l + k] += c[k];
      }
      for (int k = 0; k < RHS_KINDS; ++k) {
        F.rhs_off[RHS_KINDS * l + k] = (int)tot;
        tot += F.rhs_cap[RHS_KINDS * l + k];
      }
    }
    if (tot > INT32_MAX) throw std::runtime_error("multi-RHS task lists exceed 2^31 entries");
    F.d_rhs_tasks = F.rhs_arena.alloc<int2>(std::max<long long>(1, tot));
    F.d_rhs_off = F.rhs_arena.alloc<int>(F.rhs_off.size());
    F.d_rhs_cnt = F.rhs_arena.alloc<int>(F.rhs_off.size());
    F.d_level_first = F.rhs_arena.alloc<int>(level_first.size());
    ICR_HIP(hipMemcpyAsync(F.d_rhs_off, F.rhs_off.data(), F.rhs_off.size() * sizeof(int), hipMemcpyHostToDevice,
                           s->stream));
    ICR_HIP(hipMemcpyAsync(F.d_level_first, level_first.data(), level_first.size() * sizeof(int),
                           hipMemcpyHostToDevice, s->stream));
  }
  const long long m = 3LL * nc;
  F.d_Wp = F.rhs_arena.alloc<double>(m * m);
  F.d_keys = F.rhs_arena.alloc<int>(nc);
  F.d_order = F.rhs_arena.alloc<int>(nc);
  F.d_pos = F.rhs_arena.alloc<int>(nc);
  F.d_lohi = F.rhs_arena.alloc<int>(3LL * F.sup.size());
  F.d_fpos = F.rhs_arena.alloc<double>(3LL * nc);
  F.d_cerr = F.rhs_arena.alloc<int>(1);
  {
    // Z f tasks: one per (supernode, 64-row block, column chunk of ZF_K), the
    // chunk-0 tasks first (they also do the sums); partials per supernode at
    // off_s + chunk * n3 + row
    std::vector<int4> first, rest;
    long long off = 0;
    for (int i = 0; i < (int)F.sup.size(); ++i) {
      const SupDev &d = F.sup[i];
      const int n3 = 3 * d.ncol, nch = std::max(1, cdiv(d.rmax, ZF_K));
      for (int i0 = 0; i0 < n3; i0 += GV_R)
        for (int ch = 0; ch < nch; ++ch) (ch == 0 ? first : rest).push_back(make_int4(i, i0, ch * ZF_K, (int)off));
      off += (long long)n3 * nch;
    }
    F.n_zf_sum_tasks = (int)first.size();
    first.insert(first.end(), rest.begin(), rest.end());
    F.n_zf_tasks = (int)first.size();
    F.d_zf_tasks = F.rhs_arena.alloc<int4>(first.size());
    F.d_zf_part = F.rhs_arena.alloc<double>(std::max<long long>(1, off));
    ICR_HIP(hipMemcpyAsync(F.d_zf_tasks, first.data(), first.size() * sizeof(int4), hipMemcpyHostToDevice,
                           s->stream));
  }
  ICR_HIP(hipMemcpyAsync(F.d_sup, F.sup.data(), F.sup.size() * sizeof(SupDev), hipMemcpyHostToDevice, s->stream));
  ICR_HIP(hipStreamSynchronize(s->stream));
  F.nc_cap = nc;
}

namespace {

// Contact order and the task lists of every tree level (shared by the FP64
// and the mixed-precision builds).
void rhs_prepare(icr_scene *s, int nc, const int *node_ids, bool validate) {
  auto &F = s->fac;
  hipStream_t st = s->stream;
  const int nsup = (int)F.sup.size();
  const long long m = 3LL * nc;
  s->last_build_nc = nc;
  if (validate) ICR_HIP(hipMemsetAsync(F.d_cerr, 0, sizeof(int), st));
  k_sort_contacts<<<1, 1024, 0, st>>>(nc, s->mesh.N, nsup, node_ids, F.d_sup_of_node, s->mesh.d_fixed, F.d_keys,
                                      F.d_order, F.d_pos, F.d_cerr);
  ICR_LAUNCH_CHECK();
  const int nlev = (int)F.levels.size();
  k_rhs_plan<<<nlev, PLAN_NT, 0, st>>>(nc, F.d_level_first, F.d_level_sup, F.d_sup, F.d_keys, F.d_lohi, F.d_rhs_off,
                                      F.d_rhs_cnt, F.d_rhs_tasks);
  ICR_LAUNCH_CHECK();
  k_fill<<<1024, 256, 0, st>>>(m * m, 0.0, F.d_Wp);
  ICR_LAUNCH_CHECK();
}

// Launch geometry of a product: its list's capacity (one workgroup per task;
// the hardware keeps scheduling workgroups of both streams' launches).
struct RhsLists {
  const Factor &F;
  unsigned grid(int l, int k) const { return (unsigned)std::max(1, F.rhs_cap[RHS_KINDS * l + k]); }
  const int2 *list(int l, int k) const { return F.d_rhs_tasks + F.rhs_off[RHS_KINDS * l + k]; }
  const int *count(int l, int k) const { return F.d_rhs_cnt + RHS_KINDS * l + k; }
  bool any(int l, int k) const { return F.rhs_cap[RHS_KINDS * l + k] > 0; }
};

// Wp (mirrored) -> W_H in contact order, FP64 or FP32.
template <class TW>
void wh_finish(icr_scene *s, int nc, TW *WH) {
  auto &F = s->fac;
  const long long m = 3LL * nc;
  const int nt = cdiv(m, 64);
  k_wp_mirror<<<nt * (nt + 1) / 2, 256, 0, s->stream>>>((int)m, F.d_Wp);
  ICR_LAUNCH_CHECK();
  k_wh_unpermute<TW><<<(unsigned)m, 256, 0, s->stream>>>(nc, F.d_pos, F.d_Wp, WH);
  ICR_LAUNCH_CHECK();
}

// One forward sweep over the tree levels in FP32 (the bulk solve of the
// mixed-precision build): X32 assembled from the unit columns (R null) or
// from the residual R and the children, Z32 = L_ss^-1 X32 with its FP64 copy
// stored (z64 = 1) or added (z64 = 2) into Z, X32 below rows -= L_21 Z32.
void forward_fp32(icr_scene *s, const int *node_ids, const double *R, int z64) {
  auto &F = s->fac;
  hipStream_t st = s->stream;
  RhsLists L{F};
  for (int l = 0; l < (int)F.levels.size(); ++l) {
    if (!L.any(l, RT_ASM)) continue;
    k_rhs_assemble<float><<<L.grid(l, RT_ASM), 256, 0, st>>>(F.d_sup, L.list(l, RT_ASM), L.count(l, RT_ASM),
                                                             F.d_child, F.d_invmap_off, F.d_invmap, F.d_lohi,
                                                             F.d_order, node_ids, F.d_iperm, nullptr, R, F.d_X32);
    ICR_LAUNCH_CHECK();
    k_rhs_diag<AccS32><<<L.grid(l, RT_DIAG), 256, 0, st>>>(F.d_sup, L.list(l, RT_DIAG), L.count(l, RT_DIAG),
                                                           F.d_lohi, F.d_linv32, F.d_X32, F.d_Z32, F.d_Z, z64);
    ICR_LAUNCH_CHECK();
    if (L.any(l, RT_OFF)) {
      k_rhs_off<AccS32><<<L.grid(l, RT_OFF), 256, 0, st>>>(F.d_sup, L.list(l, RT_OFF), L.count(l, RT_OFF), F.d_lohi,
                                                           F.d_front32, F.d_Z32, F.d_X32);
      ICR_LAUNCH_CHECK();
    }
  }
}

}  // namespace

void ensure_mixed(icr_scene *s) {
  auto &F = s->fac;
  hipStream_t st = s->stream;
  if (!F.have32) {
    F.fac32_arena.release();
    F.d_front32 = F.fac32_arena.alloc<float>(F.front_elems);
    F.d_linv32 = F.fac32_arena.alloc<float>(F.linv_elems);
    k_to_float<<<2048, 256, 0, st>>>(F.front_elems, F.d_front, F.d_front32);
    ICR_LAUNCH_CHECK();
    k_to_float<<<2048, 256, 0, st>>>(F.linv_elems, F.d_linv, F.d_linv32);
    ICR_LAUNCH_CHECK();
    F.have32 = true;
  }
  if (F.mixed_cap != F.nc_cap) {
    ICR_HIP(hipStreamSynchronize(st));
    F.mixed_arena.release();
    F.d_X32 = F.mixed_arena.alloc<float>(F.x_elems);
    F.d_Z32 = F.mixed_arena.alloc<float>(F.z_elems);
    F.d_R = F.mixed_arena.alloc<double>(F.z_elems);
    F.mixed_cap = F.nc_cap;
  }
}

void build_WH_device(icr_scene *s, int nc, const int *node_ids, double *WH, bool validate, const double *frames) {
  auto &F = s->fac;
  hipStream_t st = s->stream;
  const long long m = 3LL * nc;
  rhs_prepare(s, nc, node_ids, validate);
  RhsLists L{F};
  for (int l = 0; l < (int)F.levels.size(); ++l) {
    if (!L.any(l, RT_ASM)) continue;   // no supernode of the level can hold a contact column
    k_rhs_assemble<double><<<L.grid(l, RT_ASM), 256, 0, st>>>(F.d_sup, L.list(l, RT_ASM), L.count(l, RT_ASM),
                                                              F.d_child, F.d_invmap_off, F.d_invmap, F.d_lohi,
                                                              F.d_order, node_ids, F.d_iperm, frames, nullptr,
                                                              F.d_X);
    ICR_LAUNCH_CHECK();
    k_rhs_diag<AccS><<<L.grid(l, RT_DIAG), 256, 0, st>>>(F.d_sup, L.list(l, RT_DIAG), L.count(l, RT_DIAG), F.d_lohi,
                                                         F.d_linv, F.d_X, F.d_Z, nullptr, 0);
    ICR_LAUNCH_CHECK();
    // Z of this level is final: its W_H products go to the side stream (they
    // read Z and write Wp only, which nothing on the main stream touches
    // until the join)
    hipStream_t sy = st;
    if (s->overlap) {
      ICR_HIP(hipEventRecord(s->ev_fork, st));
      ICR_HIP(hipStreamWaitEvent(s->side, s->ev_fork, 0));
      sy = s->side;
    }
    k_rhs_syrk<AccS><<<L.grid(l, RT_SYRK), 256, 0, sy>>>(F.d_sup, L.list(l, RT_SYRK), L.count(l, RT_SYRK), F.d_lohi,
                                                         F.d_Z, (int)m, F.d_Wp);
    ICR_LAUNCH_CHECK();
    if (L.any(l, RT_OFF)) {
      k_rhs_off<AccS><<<L.grid(l, RT_OFF), 256, 0, st>>>(F.d_sup, L.list(l, RT_OFF), L.count(l, RT_OFF), F.d_lohi,
                                                         F.d_front, F.d_Z, F.d_X);
      ICR_LAUNCH_CHECK();
    }
  }
  if (s->overlap) {
    ICR_HIP(hipEventRecord(s->ev_join, s->side));
    ICR_HIP(hipStreamWaitEvent(st, s->ev_join, 0));
  }
  wh_finish<double>(s, nc, WH);
}

void build_WH_mixed(icr_scene *s, int nc, const int *node_ids, int refine, float *WH32, double *WH64) {
  auto &F = s->fac;
  hipStream_t st = s->stream;
  const long long m = 3LL * nc;
  rhs_prepare(s, nc, node_ids, false);
  RhsLists L{F};
  forward_fp32(s, node_ids, nullptr, 1);   // Z32 and its FP64 copy Z
  for (int it = 0; it < refine; ++it) {
    // FP64 residual of L Z = P H^T on every supernode's rows, level by level
    for (int l = 0; l < (int)F.levels.size(); ++l) {
      if (!L.any(l, RT_ASM)) continue;
      k_rhs_assemble<double><<<L.grid(l, RT_ASM), 256, 0, st>>>(F.d_sup, L.list(l, RT_ASM), L.count(l, RT_ASM),
                                                                F.d_child, F.d_invmap_off, F.d_invmap, F.d_lohi,
                                                                F.d_order, node_ids, F.d_iperm, nullptr, nullptr,
                                                                F.d_X);
      ICR_LAUNCH_CHECK();
      k_rhs_resid<AccS><<<L.grid(l, RT_DIAG), 256, 0, st>>>(F.d_sup, L.list(l, RT_DIAG), L.count(l, RT_DIAG),
                                                            F.d_lohi, F.d_front, F.d_X, F.d_Z, F.d_R);
      ICR_LAUNCH_CHECK();
      if (L.any(l, RT_OFF)) {
        k_rhs_off<AccS><<<L.grid(l, RT_OFF), 256, 0, st>>>(F.d_sup, L.list(l, RT_OFF), L.count(l, RT_OFF), F.d_lohi,
                                                           F.d_front, F.d_Z, F.d_X);
        ICR_LAUNCH_CHECK();
      }
    }
    forward_fp32(s, node_ids, F.d_R, 2);   // Z += L^-1 R (FP32 solve of the correction)
  }
  // W_H = Z^T Z in FP64 from the refined Z
  for (int l = 0; l < (int)F.levels.size(); ++l) {
    if (!L.any(l, RT_ASM)) continue;
    k_rhs_syrk<AccS><<<L.grid(l, RT_SYRK), 256, 0, st>>>(F.d_sup, L.list(l, RT_SYRK), L.count(l, RT_SYRK), F.d_lohi,
                                                         F.d_Z, (int)m, F.d_Wp);
    ICR_LAUNCH_CHECK();
  }
  const int nt = cdiv(m, 64);
  k_wp_mirror<<<nt * (nt + 1) / 2, 256, 0, st>>>((int)m, F.d_Wp);
  ICR_LAUNCH_CHECK();
  if (WH32) {
    k_wh_unpermute<float><<<(unsigned)m, 256, 0, st>>>(nc, F.d_pos, F.d_Wp, WH32);
    ICR_LAUNCH_CHECK();
  }
  if (WH64) {
    k_wh_unpermute<double><<<(unsigned)m, 256, 0, st>>>(nc, F.d_pos, F.d_Wp, WH64);
    ICR_LAUNCH_CHECK();
  }
}

}  // namespace icr
