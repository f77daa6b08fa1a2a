// Contact side of the time step: selection of the contacts at the free motion
// (stand-in for collision detection, Sec. "Contact generation"), frames and
// gaps (Eq. 7, 10, 26), the fast compliance update W = C W_H C^T (Eq. 28),
// projected Gauss-Seidel (Eq. 18-19, Algorithm 1), and the proximity update
// p_k = p_free + h^2 W_H C_k^T lambda_k (Eq. 31).
#include <hip/hip_cooperative_groups.h>

#include <algorithm>
#include <mutex>

#include "scene.hpp"

namespace icr {

namespace {

__device__ inline unsigned long long sortable(double x) {
  unsigned long long b = (unsigned long long)__double_as_longlong(x);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__device__ double signed_distance(const icr_obstacle &o, double t, const double p[3], double nrm[3]) {
#pragma clang fp contract(off)
  double c[3] = {o.c0[0] + o.vel[0] * t, o.c0[1] + o.vel[1] * t, o.c0[2] + o.vel[2] * t};
  double r0 = p[0] - c[0], r1 = p[1] - c[1], r2 = p[2] - c[2];
  if (o.kind == 1) {
    double dist = sqrt(r0 * r0 + r1 * r1 + r2 * r2);
    nrm[0] = r0 / dist;
    nrm[1] = r1 / dist;
    nrm[2] = r2 / dist;
    return dist - o.radius;
  }
  nrm[0] = o.normal[0];
  nrm[1] = o.normal[1];
  nrm[2] = o.normal[2];
  return r0 * o.normal[0] + r1 * o.normal[1] + r2 * o.normal[2];
}

// Exclusive prefix sum of one int per thread over a 1024-thread block.
__device__ int block_excl_scan_1024(int v, int *wsum) {
  const int ln = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int x = v;
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(x, o, 64);
    if (ln >= o) x += t;
  }
  if (ln == 63) wsum[wv] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int w = 0; w < 16; ++w) {
      const int t = wsum[w];
      wsum[w] = acc;
      acc += t;
    }
  }
  __syncthreads();
  const int r = wsum[wv] + x - v;
  __syncthreads();
  return r;
}

// Keep the K candidates with smallest (distance, node id) at q_free, in
// ascending node id; gather mu, p_free = H q_free, p_start = H q, warm start.
// The candidate list is ascending by node id (sorted when it is set).  The
// K-th smallest distance key T is found by an MSB-first radix select (8 bits
// per pass, 256-bin histograms in LDS); the contacts are the candidates with
// key < T and the lowest-id ones with key == T, placed by an exclusive scan
// of the selection flags in list order.  Thread t holds list entries
// 4t .. 4t + 3.
constexpr int SEL_PER = 4;   // 4096 candidates at most
__global__ __launch_bounds__(1024) void k_select(int ncand, const int *__restrict__ cand,
                                                 const double *__restrict__ qf, const double *__restrict__ q,
                                                 const StepCtx *__restrict__ ctx, int K,
                                                 const double *__restrict__ mu_node,
                                                 const double *__restrict__ node_force, int *__restrict__ nodes_c,
                                                 double *__restrict__ mu_c, double *__restrict__ pfree,
                                                 double *__restrict__ pstart, double *__restrict__ finit) {
  __shared__ unsigned long long key[1024 * SEL_PER];
  __shared__ int hist[256];
  __shared__ int wsum[16];
  __shared__ unsigned long long s_prefix;
  __shared__ int s_rank;
  const int tid = threadIdx.x, ln = tid & 63, wv = tid >> 6;
  const icr_obstacle obs = ctx->obs;
  const double t1 = ctx->t0 + ctx->h;
#pragma unroll
  for (int e = 0; e < SEL_PER; ++e) {
    const int i = SEL_PER * tid + e;
    unsigned long long kv = ~0ull;
    if (i < ncand) {
      const int v = cand[i];
      double p[3] = {qf[3 * v], qf[3 * v + 1], qf[3 * v + 2]}, nrm[3];
      kv = sortable(signed_distance(obs, t1, p, nrm));
    }
    key[i] = kv;
  }
  if (tid == 0) {
    s_prefix = 0ull;
    s_rank = K;   // rank (1-based) of the sought key among those matching the prefix
  }
  unsigned long long mask = 0ull;
  for (int shift = 56; shift >= 0; shift -= 8) {
    for (int b = tid; b < 256; b += 1024) hist[b] = 0;
    __syncthreads();
    const unsigned long long prefix = s_prefix;
#pragma unroll
    for (int e = 0; e < SEL_PER; ++e) {
      const int i = SEL_PER * tid + e;
      if (i < ncand && (key[i] & mask) == prefix) atomicAdd(&hist[(int)((key[i] >> shift) & 255ull)], 1);
    }
    __syncthreads();
    if (wv == 0) {
      const int c0 = hist[4 * ln], c1 = hist[4 * ln + 1], c2 = hist[4 * ln + 2], c3 = hist[4 * ln + 3];
      const int tot = c0 + c1 + c2 + c3;
      int incl = tot;
      for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(incl, o, 64);
        if (ln >= o) incl += t;
      }
      const int rank = s_rank;
      int run = incl - tot;
      const int c[4] = {c0, c1, c2, c3};
      for (int qd = 0; qd < 4; ++qd) {
        if (run < rank && rank <= run + c[qd]) {   // exactly one bin of the wave
          s_prefix = prefix | ((unsigned long long)(4 * ln + qd) << shift);
          s_rank = rank - run;
        }
        run += c[qd];
      }
    }
    __syncthreads();
    mask |= 0xffull << shift;
  }
  const unsigned long long T = s_prefix;
  const int need = s_rank;   // candidates with key == T to keep, lowest ids first
  int tf[SEL_PER], tsum = 0;
#pragma unroll
  for (int e = 0; e < SEL_PER; ++e) {
    const int i = SEL_PER * tid + e;
    tf[e] = (i < ncand && key[i] == T) ? 1 : 0;
    tsum += tf[e];
  }
  int tr = block_excl_scan_1024(tsum, wsum);
  int sf[SEL_PER], ssum = 0;
#pragma unroll
  for (int e = 0; e < SEL_PER; ++e) {
    const int i = SEL_PER * tid + e;
    sf[e] = (i < ncand && (key[i] < T || (tf[e] && tr < need))) ? 1 : 0;
    tr += tf[e];
    ssum += sf[e];
  }
  int c = block_excl_scan_1024(ssum, wsum);
#pragma unroll
  for (int e = 0; e < SEL_PER; ++e) {
    if (!sf[e]) continue;
    const int v = cand[SEL_PER * tid + e];
    nodes_c[c] = v;
    mu_c[c] = mu_node[v];
    for (int a = 0; a < 3; ++a) {
      pfree[3 * c + a] = qf[3 * v + a];
      pstart[3 * c + a] = q[3 * v + a];
      finit[3 * c + a] = node_force[3 * v + a];
    }
    ++c;
  }
}

// Frame (rows n, t1, t2: normal and axis-rule tangents) and gap delta of a
// contact at proximity pc: normal gap = signed distance at t1, tangential gap
// = relative tangential displacement over the step.
__device__ inline void contact_frame(const icr_obstacle &obs, double t0, double t1, const double pc[3],
                                     const double ps[3], double F[3][3], double delta[3]) {
  double n[3];
  double phi = signed_distance(obs, t1, pc, n);
  int ax = 0;
  double am = fabs(n[0]);
  if (fabs(n[1]) < am) {
    ax = 1;
    am = fabs(n[1]);
  }
  if (fabs(n[2]) < am) ax = 2;
  double en = n[ax];
  double ta[3] = {-en * n[0], -en * n[1], -en * n[2]};
  ta[ax] += 1.0;
  double tn = sqrt(ta[0] * ta[0] + ta[1] * ta[1] + ta[2] * ta[2]);
  ta[0] /= tn;
  ta[1] /= tn;
  ta[2] /= tn;
  double tb[3] = {n[1] * ta[2] - n[2] * ta[1], n[2] * ta[0] - n[0] * ta[2], n[0] * ta[1] - n[1] * ta[0]};
  double rel[3];
  for (int a = 0; a < 3; ++a) {
    double uo = (obs.c0[a] + obs.vel[a] * t1) - (obs.c0[a] + obs.vel[a] * t0);
    rel[a] = pc[a] - ps[a] - uo;
  }
  for (int a = 0; a < 3; ++a) {
    F[0][a] = n[a];
    F[1][a] = ta[a];
    F[2][a] = tb[a];
  }
  delta[0] = phi;
  delta[1] = ta[0] * rel[0] + ta[1] * rel[1] + ta[2] * rel[2];
  delta[2] = tb[0] * rel[0] + tb[1] * rel[1] + tb[2] * rel[2];
}

// Frame and gap of a pair contact between two bodies: the given normal n of
// the second body's surface (fixed over the step), tangents by the axis
// rule, normal gap n . p of the relative position p = x_1 - x_2, tangential
// gap = relative tangential displacement over the step.
__device__ inline void pair_frame(const double n[3], const double pc[3], const double ps[3], double F[3][3],
                                  double delta[3]) {
  int ax = 0;
  double am = fabs(n[0]);
  if (fabs(n[1]) < am) {
    ax = 1;
    am = fabs(n[1]);
  }
  if (fabs(n[2]) < am) ax = 2;
  double en = n[ax];
  double ta[3] = {-en * n[0], -en * n[1], -en * n[2]};
  ta[ax] += 1.0;
  double tn = sqrt(ta[0] * ta[0] + ta[1] * ta[1] + ta[2] * ta[2]);
  ta[0] /= tn;
  ta[1] /= tn;
  ta[2] /= tn;
  double tb[3] = {n[1] * ta[2] - n[2] * ta[1], n[2] * ta[0] - n[0] * ta[2], n[0] * ta[1] - n[1] * ta[0]};
  double rel[3] = {pc[0] - ps[0], pc[1] - ps[1], pc[2] - ps[2]};
  for (int a = 0; a < 3; ++a) {
    F[0][a] = n[a];
    F[1][a] = ta[a];
    F[2][a] = tb[a];
  }
  delta[0] = n[0] * pc[0] + n[1] * pc[1] + n[2] * pc[2];
  delta[1] = ta[0] * rel[0] + ta[1] * rel[1] + ta[2] * rel[2];
  delta[2] = tb[0] * rel[0] + tb[1] * rel[1] + tb[2] * rel[2];
}

// Frames C_k and gaps at p_{k-1}; d_k = delta - C_k (p - p_free); warm start
// lambda = C_k f with f the previous world-frame force.  The first npair
// contacts are pairs with normals pn.
__global__ void k_directions(int nc, const StepCtx *__restrict__ ctx, const double *__restrict__ p,
                             const double *__restrict__ pfree, const double *__restrict__ pstart,
                             const double *__restrict__ fprev, double *__restrict__ C, double *__restrict__ dk,
                             double *__restrict__ lam, int npair, const double *__restrict__ pn) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  const icr_obstacle obs = ctx->obs;
  const double t0 = ctx->t0, t1 = ctx->t0 + ctx->h;
  double pc[3] = {p[3 * c], p[3 * c + 1], p[3 * c + 2]};
  double ps[3] = {pstart[3 * c], pstart[3 * c + 1], pstart[3 * c + 2]};
  double F[3][3], delta[3];
  if (c < npair) {
    const double n[3] = {pn[3 * c], pn[3 * c + 1], pn[3 * c + 2]};
    pair_frame(n, pc, ps, F, delta);
  } else {
    contact_frame(obs, t0, t1, pc, ps, F, delta);
  }
  double dp[3] = {pc[0] - pfree[3 * c], pc[1] - pfree[3 * c + 1], pc[2] - pfree[3 * c + 2]};
  for (int r = 0; r < 3; ++r) {
    for (int a = 0; a < 3; ++a) C[9 * c + 3 * r + a] = F[r][a];
    dk[3 * c + r] = delta[r] - (F[r][0] * dp[0] + F[r][1] * dp[1] + F[r][2] * dp[2]);
    lam[3 * c + r] = F[r][0] * fprev[3 * c] + F[r][1] * fprev[3 * c + 1] + F[r][2] * fprev[3 * c + 2];
  }
}

// W_ab = C_a (W_H)_ab C_b^T.  Block (a, b) with a < b is computed as the
// transpose of block (b, a) from the same inputs (W_H is exactly symmetric),
// so W is exactly symmetric.
template <class TW>
__device__ __forceinline__ void update_W_block(int nc, const TW *__restrict__ WH, const double *__restrict__ C,
                                               TW *__restrict__ W, long blk) {
  const int a = (int)(blk / nc), b = (int)(blk % nc);
  const long m = 3L * nc;
  const bool lower = a >= b;
  double M[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double v = (double)WH[(3L * a + i) * m + 3L * b + j];
      if (lower)
        M[i][j] = v;
      else
        M[j][i] = v;
    }
  const double *X = C + 9L * (lower ? a : b);
  const double *Y = C + 9L * (lower ? b : a);
  double T[3][3];   // M Y^T
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) T[i][j] = M[i][0] * Y[3 * j] + M[i][1] * Y[3 * j + 1] + M[i][2] * Y[3 * j + 2];
  double R[3][3];   // X T
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) R[i][j] = X[3 * i] * T[0][j] + X[3 * i + 1] * T[1][j] + X[3 * i + 2] * T[2][j];
  // diagonal blocks: mirror the lower entries so the block is exactly symmetric
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double v;
      if (a == b)
        v = (i >= j) ? R[i][j] : R[j][i];
      else
        v = lower ? R[i][j] : R[j][i];
      W[(3L * a + i) * m + 3L * b + j] = (TW)v;
    }
}

template <class TW>
__global__ void k_update_W(int nc, const TW *__restrict__ WH, const double *__restrict__ C, TW *__restrict__ W) {
  const long blk = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (blk < (long)nc * nc) update_W_block(nc, WH, C, W, blk);
}

// ---- local solver (Signorini + Coulomb cone) --------------------------------

struct Local {
  double l[3];
  int st;
};

__device__ Local local_solve(const double w[3][3], const double d[3], double mu, int j_inner) {
  Local out;
  if (d[0] >= 0.0) {
    out.l[0] = out.l[1] = out.l[2] = 0.0;
    out.st = ICR_SEPARATE;
    return out;
  }
  // stick trial: 3x3 Cholesky solve
  double l00 = sqrt(w[0][0]);
  double l10 = w[1][0] / l00, l20 = w[2][0] / l00;
  double l11 = sqrt(w[1][1] - l10 * l10);
  double l21 = (w[2][1] - l20 * l10) / l11;
  double l22 = sqrt(w[2][2] - l20 * l20 - l21 * l21);
  double y0 = d[0] / l00;
  double y1 = (d[1] - l10 * y0) / l11;
  double y2 = (d[2] - l20 * y0 - l21 * y1) / l22;
  double x2 = y2 / l22;
  double x1 = (y1 - l21 * x2) / l11;
  double x0 = (y0 - l10 * x1 - l20 * x2) / l00;
  double ln = -x0, lt1 = -x1, lt2 = -x2;
  if (ln > 0.0 && lt1 * lt1 + lt2 * lt2 <= (mu * ln) * (mu * ln)) {
    out.l[0] = ln;
    out.l[1] = lt1;
    out.l[2] = lt2;
    out.st = ICR_STICK;
    return out;
  }
  double u0, u1;
  double nt = sqrt(lt1 * lt1 + lt2 * lt2);
  if (nt > 0.0) {
    u0 = lt1 / nt;
    u1 = lt2 / nt;
  } else {
    double ndt = sqrt(d[1] * d[1] + d[2] * d[2]);
    if (ndt > 0.0) {
      u0 = -d[1] / ndt;
      u1 = -d[2] / ndt;
    } else {
      u0 = 1.0;
      u1 = 0.0;
    }
  }
  const double kap = 0.5 * (w[1][1] + w[2][2]);
  for (int it = 0; it < j_inner; ++it) {
    double den = w[0][0] + mu * (w[0][1] * u0 + w[0][2] * u1);
    if (den <= 0.0) den = w[0][0];
    double lam_n = -d[0] / den;
    double a1 = mu * lam_n * u0, a2 = mu * lam_n * u1;
    double r1 = d[1] + w[1][0] * lam_n + (w[1][1] - kap) * a1 + w[1][2] * a2;
    double r2 = d[2] + w[2][0] * lam_n + w[2][1] * a1 + (w[2][2] - kap) * a2;
    double nr = sqrt(r1 * r1 + r2 * r2);
    if (nr > 0.0) {
      u0 = -r1 / nr;
      u1 = -r2 / nr;
    }
  }
  double den = w[0][0] + mu * (w[0][1] * u0 + w[0][2] * u1);
  if (den <= 0.0) den = w[0][0];
  double lam_n = -d[0] / den;
  out.l[0] = lam_n;
  out.l[1] = mu * lam_n * u0;
  out.l[2] = mu * lam_n * u1;
  out.st = ICR_SLIP;
  return out;
}

// 1/x and 1/sqrt(x) from the hardware estimates refined by two Newton steps
// (full double precision for the well-scaled positive values used here).
__device__ inline double frcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(fma(-x, r, 1.0), r, r);
  return fma(fma(-x, r, 1.0), r, r);
}
__device__ inline double frsqrt(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
  return fma(0.5 * y, fma(-x * y, y, 1.0), y);
}
// One Newton step only: relative error about the square of the estimate's
// (used inside the slip fixed point, whose iterates are renormalised anyway).
__device__ inline double frsqrt1(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  return fma(0.5 * y, fma(-x * y, y, 1.0), y);
}

// Per-contact record of the active-set PGS, computed once per active set from
// the symmetric 3x3 block w of h^2 W_aa and mu (kappa = (w11 + w22) / 2):
//   0-5  w00 w01 w02 w11 w12 w22      6-11 the same entries of -w^-1
//   12   mu (w11 - kappa)   13 mu (w22 - kappa)   14 mu w12
//   15   mu w01             16 mu w02             17 mu
//   18   1 if w00 > mu |(w01, w02)| with margin (then den(u) > 0 on the unit
//        circle and the slip pass needs no fallback), else 0
// FAST (a record built inside a Gauss-Seidel visit, on its dependent chain):
// the refined reciprocal for 1 / det and the margin test compared squared.
constexpr int PGS_RW = kPgsRecWidth;   // record width: 19 entries, then the contact's current force (chain)
template <bool FAST = false>
__device__ inline void make_record(const double w[3][3], double mu, double *rec) {
  const double w00 = w[0][0], w01 = w[0][1], w02 = w[0][2], w11 = w[1][1], w12 = w[1][2], w22 = w[2][2];
  const double c00 = w11 * w22 - w12 * w12, c01 = w02 * w12 - w01 * w22, c02 = w01 * w12 - w02 * w11;
  const double c11 = w00 * w22 - w02 * w02, c12 = w01 * w02 - w00 * w12, c22 = w00 * w11 - w01 * w01;
  const double det = w00 * c00 + w01 * c01 + w02 * c02;
  const double idet = FAST ? frcp(det) : 1.0 / det;
  const double kap = 0.5 * (w11 + w22);
  rec[0] = w00;
  rec[1] = w01;
  rec[2] = w02;
  rec[3] = w11;
  rec[4] = w12;
  rec[5] = w22;
  rec[6] = -(c00 * idet);
  rec[7] = -(c01 * idet);
  rec[8] = -(c02 * idet);
  rec[9] = -(c11 * idet);
  rec[10] = -(c12 * idet);
  rec[11] = -(c22 * idet);
  rec[12] = mu * (w11 - kap);
  rec[13] = mu * (w22 - kap);
  rec[14] = mu * w12;
  rec[15] = mu * w01;
  rec[16] = mu * w02;
  rec[17] = mu;
  if (FAST) {
    const double mm = 1.000001 * mu;   // w00 > mm |(w01, w02)| squared, w00 > 0
    rec[18] = (w00 > 0.0 && w00 * w00 > (mm * mm) * (w01 * w01 + w02 * w02)) ? 1.0 : 0.0;
  } else {
    rec[18] = (w00 > 1.000001 * mu * sqrt(w01 * w01 + w02 * w02)) ? 1.0 : 0.0;
  }
}

// Guarded slip pass (rare: the record's den > 0 guarantee fails, or |v| = 0
// occurred): den <= 0 replaced by w_nn as in the direct form, |v| = 0 keeps
// the direction; restarts from the same initial direction.  Out of line, so
// the chains' straight-line code keeps its registers.
struct SlipIn {
  double w00, w01, w02, mm11, mm22, mw12, mw01, mw02;   // record entries
  double d0, d1, d2, lt1, lt2, nt2;                     // gap, stick trial
  double n0, n1, n00, n01, n10, n11;                    // -v(u) = n + N u
};
__device__ __noinline__ double2 guarded_slip(const SlipIn a, int j_inner) {
  const double w00 = a.w00, w01 = a.w01, w02 = a.w02, mm11 = a.mm11, mm22 = a.mm22, mw12 = a.mw12, mw01 = a.mw01,
               mw02 = a.mw02;
  const double d[3] = {a.d0, a.d1, a.d2};
  const double lt1 = a.lt1, lt2 = a.lt2, nt2 = a.nt2;
  const double n0 = a.n0, n1 = a.n1, n00 = a.n00, n01 = a.n01, n10 = a.n10, n11 = a.n11;
  double u0, u1;
  if (nt2 > 0.0) {
    const double inv = frsqrt(nt2);
    u0 = lt1 * inv;
    u1 = lt2 * inv;
  } else {
    const double nd2 = d[1] * d[1] + d[2] * d[2];
    if (nd2 > 0.0) {
      const double inv = frsqrt(nd2);
      u0 = -d[1] * inv;
      u1 = -d[2] * inv;
    } else {
      u0 = 1.0;
      u1 = 0.0;
    }
  }
  for (int it = 0; it < j_inner; ++it) {
    const double den = fma(mw01, u0, fma(mw02, u1, w00));
    double v0, v1;
    if (den > 0.0) {
      v0 = fma(n00, u0, fma(n01, u1, n0));
      v1 = fma(n10, u0, fma(n11, u1, n1));
    } else {
      const double e1 = fma(mm11, u0, fma(mw12, u1, w01)), e2 = fma(mw12, u0, fma(mm22, u1, w02));
      v0 = fma(d[0], e1, -w00 * d[1]);
      v1 = fma(d[0], e2, -w00 * d[2]);
    }
    const double s2 = v0 * v0 + v1 * v1;
    if (s2 > 0.0) {
      const double inv = frsqrt(s2);
      u0 = v0 * inv;
      u1 = v1 * inv;
    }
  }
  return make_double2(u0, u1);
}

// Same branches and fixed point as local_solve, from the record: stick trial
// by the precomputed inverse, refined reciprocals instead of divisions, and
// the slip pass on the direction u alone.  With den(u) > 0 the tangential
// residual r = d_t + lam_n(u) e(u), lam_n = -d_n / den(u),
// e(u) = w_tn + mu (W_tt - kappa I) u, is parallel to
//   v(u) = den(u) d_t - d_n e(u) = c + G u,
// an affine map of u, so a pass is u <- -v / |v| (same iterates up to
// rounding).  Every VALU instruction of the single issuing wave costs the
// same whatever its dependences, so the pass is kept to 14 of them.
// J = 8: the default pass count, straight-line; J = 0: j_inner passes in a loop.
template <int J>
__device__ Local local_solve_rec(const double *rc, const double d[3], int j_inner) {
  Local out;
  if (d[0] >= 0.0) {
    out.l[0] = out.l[1] = out.l[2] = 0.0;
    out.st = ICR_SEPARATE;
    return out;
  }
  const double w00 = rc[0], w01 = rc[1], w02 = rc[2];
  const double mm11 = rc[12], mm22 = rc[13], mw12 = rc[14], mw01 = rc[15], mw02 = rc[16], mu = rc[17];
  // the record holds -w^-1: the stick trial lambda = -w^-1 d without a negation
  const double ln = rc[6] * d[0] + rc[7] * d[1] + rc[8] * d[2];
  const double lt1 = rc[7] * d[0] + rc[9] * d[1] + rc[10] * d[2];
  const double lt2 = rc[8] * d[0] + rc[10] * d[1] + rc[11] * d[2];
  const double nt2 = lt1 * lt1 + lt2 * lt2;
  if (ln > 0.0 && nt2 <= (mu * ln) * (mu * ln)) {
    out.l[0] = ln;
    out.l[1] = lt1;
    out.l[2] = lt2;
    out.st = ICR_STICK;
    return out;
  }
  double u0, u1;
  if (nt2 > 0.0) {
    const double inv = frsqrt(nt2);
    u0 = lt1 * inv;
    u1 = lt2 * inv;
  } else {
    const double nd2 = d[1] * d[1] + d[2] * d[2];
    if (nd2 > 0.0) {
      const double inv = frsqrt(nd2);
      u0 = -d[1] * inv;
      u1 = -d[2] * inv;
    } else {
      u0 = 1.0;
      u1 = 0.0;
    }
  }
  // -v(u) = n + N u
  const double n0 = fma(d[0], w01, -w00 * d[1]), n1 = fma(d[0], w02, -w00 * d[2]);
  const double n00 = fma(d[0], mm11, -d[1] * mw01), n01 = fma(d[0], mw12, -d[1] * mw02);
  const double n10 = fma(d[0], mw12, -d[2] * mw01), n11 = fma(d[0], mm22, -d[2] * mw02);
  bool safe = rc[18] != 0.0;
  if (safe) {
    auto pass = [&]() {
      const double v0 = fma(n00, u0, fma(n01, u1, n0));
      const double v1 = fma(n10, u0, fma(n11, u1, n1));
      const double inv = frsqrt1(fma(v0, v0, v1 * v1));
      u0 = v0 * inv;
      u1 = v1 * inv;
    };
    if constexpr (J == 8) {   // the default count: straight-line passes, no loop branch
#pragma unroll
      for (int it = 0; it < 8; ++it) pass();
    } else {
      for (int it = 0; it < j_inner; ++it) pass();
    }
    safe = (u0 == u0) && (u1 == u1);   // |v| = 0 (a NaN) takes the guarded pass below
  }
  if (!safe) {
    const SlipIn a{w00, w01, w02, mm11, mm22, mw12, mw01, mw02, d[0], d[1], d[2], lt1, lt2, nt2,
                   n0, n1, n00, n01, n10, n11};
    const double2 u = guarded_slip(a, j_inner);
    u0 = u.x;
    u1 = u.y;
  }
  double den = fma(mw01, u0, fma(mw02, u1, w00));
  if (den <= 0.0) den = w00;
  const double lam_n = -d[0] * frcp(den);
  const double mln = mu * lam_n;
  out.l[0] = lam_n;
  out.l[1] = mln * u0;
  out.l[2] = mln * u1;
  out.st = ICR_SLIP;
  return out;
}

// Deterministic block reduction of one double (1024 threads).
__device__ double block_sum(double v, double *red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
  return s;   // valid in thread 0
}

// Deterministic block reductions over the active-set kernel's threads (valid
// in thread 0): three sums at once, and a minimum.
__device__ void block_sum3(double &a, double &b, double &c, double *red) {
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o, 64);
    b += __shfl_xor(b, o, 64);
    c += __shfl_xor(c, o, 64);
  }
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, nw = (int)(blockDim.x >> 6);
  __syncthreads();
  if (l == 0) {
    red[w] = a;
    red[16 + w] = b;
    red[32 + w] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    a = b = c = 0.0;
    for (int i = 0; i < nw; ++i) {
      a += red[i];
      b += red[16 + i];
      c += red[32 + i];
    }
  }
}
__device__ double block_min(double v, double *red) {
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, nw = (int)(blockDim.x >> 6);
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  double r = INFINITY;
  if (threadIdx.x == 0)
    for (int i = 0; i < nw; ++i) r = fmin(r, red[i]);
  return r;
}

// g0 = d + h^2 W lambda0, one wave per row (the PGS start state).
// y = x0 + h2 M v for a symmetric m x m row-major M (m = 3 nc) and a vector v
// that is non-zero on few contacts (3-blocks of v): by symmetry
// (M v)_i = sum over contacts k with a non-zero block of M[3k+a][i] v[3k+a],
// so only those rows of M are read, each contiguous in the output index i.
// A skipped term is an exact zero, so only the summation order differs from
// the dense product.  Every block compacts the non-zero contacts (ascending,
// SG_CHUNK at a time) into LDS, then its waves split that list over the same
// 64 outputs and add their partial sums in a fixed order.
// World-frame force of contact c from its frame rows and force components.
__device__ inline double world_force(const double *__restrict__ C, const double *__restrict__ lam, long c, int a) {
  const double *R = C + 9 * c;
  return R[a] * lam[3 * c] + R[3 + a] * lam[3 * c + 1] + R[6 + a] * lam[3 * c + 2];
}

constexpr int SG_NT = 512;
constexpr int SG_NW = SG_NT / 64;
constexpr int SG_CHUNK = 2048;
__device__ inline bool block_nonzero(const double *__restrict__ v, long c) {
  return (v[3 * c] != 0.0) | (v[3 * c + 1] != 0.0) | (v[3 * c + 2] != 0.0);
}
// With C given, the vector is the world-frame force f = C^T lambda of the
// contacts (v is then ignored): every block forms the entries it needs from
// C and lambda, and block 0 also writes f for all contacts to fout.
template <class TM>
__global__ __launch_bounds__(SG_NT) void k_sym_gemv_sparse(int nc, const TM *__restrict__ M,
                                                           const double *__restrict__ x0,
                                                           const double *__restrict__ v, double h2,
                                                           double *__restrict__ y, const double *__restrict__ C,
                                                           const double *__restrict__ lam,
                                                           double *__restrict__ fout) {
  __shared__ int list[SG_CHUNK];
  __shared__ double fl[3 * SG_CHUNK];   // world forces of the listed contacts (with C)
  __shared__ int wsum[SG_NW];
  __shared__ double part[SG_NW][64];
  const int tid = threadIdx.x, wv = tid >> 6, ln = tid & 63;
  const long m = 3L * nc;
  const long i = (long)blockIdx.x * 64 + ln;
  const double *nzv = C ? lam : v;   // same zero blocks: C is a rotation
  if (C && blockIdx.x == 0)
    for (long e = tid; e < m; e += SG_NT) fout[e] = world_force(C, lam, e / 3, (int)(e % 3));
  double s = 0.0;
  for (int c0 = 0; c0 < nc; c0 += SG_CHUNK) {
    const int cn = min(SG_CHUNK, nc - c0);
    const int per = (cn + SG_NT - 1) / SG_NT;   // contiguous contacts per thread
    const int lo = c0 + min(cn, tid * per), hi = c0 + min(cn, (tid + 1) * per);
    int cnt = 0;
    for (int c = lo; c < hi; ++c) cnt += block_nonzero(nzv, c) ? 1 : 0;
    int incl = cnt;   // inclusive scan over the wave, then over the waves
    for (int o = 1; o < 64; o <<= 1) {
      const int t = __shfl_up(incl, o, 64);
      if (ln >= o) incl += t;
    }
    if (ln == 63) wsum[wv] = incl;
    __syncthreads();
    int pos = incl - cnt, total = 0;
    for (int w = 0; w < SG_NW; ++w) {
      pos += (w < wv) ? wsum[w] : 0;
      total += wsum[w];
    }
    for (int c = lo; c < hi; ++c)
      if (block_nonzero(nzv, c)) list[pos++] = c;
    __syncthreads();
    if (C) {
      for (int e = tid; e < 3 * total; e += SG_NT) fl[e] = world_force(C, lam, list[e / 3], e % 3);
      __syncthreads();
    }
    if (i < m) {
#pragma unroll 4
      for (int q = wv; q < total; q += SG_NW) {
        const long r = 3L * list[q];
        const double v0 = C ? fl[3 * q] : v[r], v1 = C ? fl[3 * q + 1] : v[r + 1], v2 = C ? fl[3 * q + 2] : v[r + 2];
        s = fma((double)M[r * m + i], v0, s);
        s = fma((double)M[(r + 1) * m + i], v1, s);
        s = fma((double)M[(r + 2) * m + i], v2, s);
      }
    }
    __syncthreads();   // list and wsum are rewritten by the next chunk
  }
  part[wv][ln] = s;
  __syncthreads();
  if (wv == 0 && i < m) {
    double t = 0.0;
    for (int w = 0; w < SG_NW; ++w) t += part[w][ln];
    y[i] = x0[i] + h2 * t;
  }
}

// Single-workgroup PGS.  g = d + W~ lambda (all contacts, own term included)
// lives in LDS; for contact a: d_a = g_a - W~_aa lambda_a, local solve, then
// g += W~[:, a] (lambda_new - lambda_old), read from rows of the exactly
// symmetric W.  A contact whose force is zero and whose gap g_n is >= 0 is a
// no-op of Gauss-Seidel (it stays separated and changes nothing), so wave 0
// scans 64 contacts at a time with a ballot and jumps to the first contact
// that can change; the iterates are those of the sequential sweep.
constexpr int PGS_MAX_NC = 4096;
// dynamic LDS of k_pgs_single: g[3 nc] doubles, then nz[nc] bytes
__host__ __device__ inline size_t pgs_single_lds(int nc) { return (size_t)nc * (3 * sizeof(double) + 1); }
template <class TW>
__global__ __launch_bounds__(1024) void k_pgs_single(int nc, const TW *__restrict__ W,
                                                     const double *__restrict__ d, const double *__restrict__ g0,
                                                     const double *__restrict__ mu, double h2,
                                                     double *__restrict__ lam, int8_t *__restrict__ status,
                                                     int max_sweeps, double tol, int j_inner,
                                                     int *__restrict__ sweeps_out, double *__restrict__ eps_out,
                                                     const int *__restrict__ ctl) {
  extern __shared__ double lds_g[];
  double *g = lds_g;
  unsigned char *nz = reinterpret_cast<unsigned char *>(lds_g + 3 * nc);
  __shared__ double bc[3];
  __shared__ double red[16];
  __shared__ int ctl_s;
  __shared__ int stop;
  // resume mode: continue where the active-set kernel handed over (or do nothing)
  int first_sweep = 0;
  if (ctl != nullptr) {
    if (ctl[0] == 0) return;
    first_sweep = ctl[1];
  }
  const int m = 3 * nc;
  const int tid = threadIdx.x, wv = tid >> 6, ln = tid & 63;
  if (g0 != nullptr) {
    for (int i = tid; i < m; i += 1024) g[i] = g0[i];
  } else {
    for (int i = wv; i < m; i += 16) {
      double sacc = 0.0;
      for (int j = ln; j < m; j += 64) sacc = fma((double)W[(long)i * m + j], lam[j], sacc);
      for (int o = 32; o > 0; o >>= 1) sacc += __shfl_xor(sacc, o, 64);
      if (ln == 0) g[i] = d[i] + h2 * sacc;
    }
  }
  for (int c = tid; c < nc; c += 1024)
    nz[c] = (lam[3 * c] != 0.0 || lam[3 * c + 1] != 0.0 || lam[3 * c + 2] != 0.0) ? 1 : 0;
  if (tid == 0) stop = 0;
  __syncthreads();
  double dsum = 0.0;   // wave 0: sum of squared changes in this sweep
  int sweep = 0;
  double eps = 0.0;
  for (sweep = first_sweep; sweep < max_sweeps; ++sweep) {
    dsum = 0.0;
    int a = 0;
    while (true) {
      if (wv == 0) {
        int next = nc;
        while (a < nc) {
          const int c = a + ln;
          const bool active = (c < nc) && (nz[c] != 0 || g[3 * c] < 0.0);
          const unsigned long long bal = __ballot(active);
          if (bal == 0ull) {
            if (c < nc) status[c] = (int8_t)ICR_SEPARATE;
            a += 64;
            continue;
          }
          const int first = __ffsll((long long)bal) - 1;
          if (ln < first && c < nc) status[c] = (int8_t)ICR_SEPARATE;
          next = a + first;
          break;
        }
        if (next < nc) {
          // every lane of wave 0 runs the local solve on the same data
          double w[3][3], lo[3], dd[3];
          for (int i = 0; i < 3; ++i) {
            lo[i] = lam[3 * next + i];
            for (int j = 0; j < 3; ++j) w[i][j] = h2 * (double)W[(3L * next + i) * m + 3L * next + j];
          }
          for (int i = 0; i < 3; ++i)
            dd[i] = g[3 * next + i] - (w[i][0] * lo[0] + w[i][1] * lo[1] + w[i][2] * lo[2]);
          Local r = local_solve(w, dd, mu[next], j_inner);
          double dl[3];
          for (int i = 0; i < 3; ++i) {
            dl[i] = r.l[i] - lo[i];
            dsum += dl[i] * dl[i];
          }
          if (ln == 0) {
            for (int i = 0; i < 3; ++i) {
              bc[i] = dl[i];
              lam[3 * next + i] = r.l[i];
            }
            status[next] = (int8_t)r.st;
            nz[next] = (r.l[0] != 0.0 || r.l[1] != 0.0 || r.l[2] != 0.0) ? 1 : 0;
          }
        }
        if (ln == 0) ctl_s = next;
      }
      __syncthreads();
      const int cur = ctl_s;
      if (cur >= nc) break;
      const double d0 = bc[0], d1 = bc[1], d2 = bc[2];
      if (d0 != 0.0 || d1 != 0.0 || d2 != 0.0) {
        const TW *r0 = W + (3L * cur) * m;
        for (int i = tid; i < m; i += 1024)
          g[i] += h2 * ((double)r0[i] * d0 + (double)r0[m + i] * d1 + (double)r0[2L * m + i] * d2);
      }
      __syncthreads();
      a = cur + 1;
    }
    // eps = |lam_i - lam_{i-1}| / |lam_i|
    double part = 0.0;
    for (int i = tid; i < m; i += 1024) part += lam[i] * lam[i];
    __threadfence_block();
    double nl2 = block_sum(part, red);
    if (tid == 0) {
      double diff = sqrt(dsum), nl = sqrt(nl2);
      eps = nl > 0.0 ? diff / nl : (diff == 0.0 ? 0.0 : INFINITY);
      stop = (eps <= tol) ? 1 : 0;
    }
    __syncthreads();
    if (stop) {
      ++sweep;
      break;
    }
  }
  if (tid == 0) {
    *sweeps_out = sweep;
    *eps_out = eps;
  }
}

// Gauss-Seidel with the directions updated before every local solve (the
// per-constraint variant of the results section), one workgroup.  The current
// proximity P = p_free + h^2 W_H f of every contact (world frame) lives in
// LDS.  At contact a's turn: frame C_a and gap delta at P_a, block
// W~_aa = h^2 C_a W_H,aa C_a^T, gap without the own force
// d = delta - W~_aa C_a f_a (the linearisation of Algorithm 3 at P_a), local
// solve, f_a = C_a^T lambda_a, then P += h^2 W_H[:, a] (f_a - f_a^old) from
// the rows of the exactly symmetric W_H.  A contact with no force and a
// non-negative normal gap is a no-op; wave 0 finds the next contact that can
// change 64 at a time and writes the frames of the skipped ones.
__host__ __device__ inline size_t pgs_pc_lds(int nc) { return (size_t)nc * 3 * sizeof(double); }
__global__ __launch_bounds__(1024) void k_pgs_pc(int nc, const StepCtx *__restrict__ ctx,
                                                 const double *__restrict__ WH, const double *__restrict__ pin,
                                                 const double *__restrict__ pstart, const double *__restrict__ mu,
                                                 double h2, double *__restrict__ f, double *__restrict__ C,
                                                 double *__restrict__ lam, int8_t *__restrict__ status,
                                                 int max_sweeps, double tol, int j_inner, int *__restrict__ sweeps_out,
                                                 double *__restrict__ eps_out, const int *__restrict__ ctl) {
  // resume mode: continue where the register-chain kernel handed over (or
  // do nothing); pin then holds the proximity of the hand-over state
  int first_sweep = 0;
  if (ctl != nullptr) {
    if (ctl[0] == 0) return;
    first_sweep = ctl[1];
  }
  extern __shared__ double lds_P[];
  double *P = lds_P;
  __shared__ double bc[3];
  __shared__ double red[16];
  __shared__ int ctl_s;
  __shared__ int stop;
  const int m = 3 * nc;
  const int tid = threadIdx.x, wv = tid >> 6, ln = tid & 63;
  const icr_obstacle obs = ctx->obs;
  const double t0 = ctx->t0, t1 = ctx->t0 + ctx->h;
  for (int i = tid; i < m; i += 1024) P[i] = pin[i];
  if (tid == 0) stop = 0;
  __syncthreads();
  int sweep = 0;
  double eps = 0.0, dsum = 0.0;
  for (sweep = first_sweep; sweep < max_sweeps; ++sweep) {
    dsum = 0.0;
    int a = 0;
    while (true) {
      if (wv == 0) {
        int next = nc;
        while (a < nc) {
          const int c = a + ln;
          bool active = false;
          double Fc[3][3], dc[3];
          if (c < nc) {
            const double pc[3] = {P[3 * c], P[3 * c + 1], P[3 * c + 2]};
            const double ps[3] = {pstart[3 * c], pstart[3 * c + 1], pstart[3 * c + 2]};
            contact_frame(obs, t0, t1, pc, ps, Fc, dc);
            active = f[3 * c] != 0.0 || f[3 * c + 1] != 0.0 || f[3 * c + 2] != 0.0 || dc[0] < 0.0;
          }
          const unsigned long long bal = __ballot(active);
          const int first = bal ? __ffsll((long long)bal) - 1 : 64;
          if (c < nc && ln < first) {   // skipped: separate, frame at its (unchanged) proximity
            for (int r = 0; r < 3; ++r) {
              for (int q = 0; q < 3; ++q) C[9L * c + 3 * r + q] = Fc[r][q];
              lam[3 * c + r] = 0.0;
            }
            status[c] = (int8_t)ICR_SEPARATE;
          }
          if (bal == 0ull) {
            a += 64;
            continue;
          }
          next = a + first;
          break;
        }
        if (next < nc) {
          // every lane of wave 0 runs the local solve on the same data
          const double pc[3] = {P[3 * next], P[3 * next + 1], P[3 * next + 2]};
          const double ps[3] = {pstart[3 * next], pstart[3 * next + 1], pstart[3 * next + 2]};
          double F[3][3], delta[3];
          contact_frame(obs, t0, t1, pc, ps, F, delta);
          double B[3][3];   // W_H,aa C_a^T
          for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
              const double *wr = WH + (3L * next + i) * m + 3L * next;
              B[i][j] = wr[0] * F[j][0] + wr[1] * F[j][1] + wr[2] * F[j][2];
            }
          double w[3][3];
          for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) w[i][j] = h2 * (F[i][0] * B[0][j] + F[i][1] * B[1][j] + F[i][2] * B[2][j]);
          for (int i = 0; i < 3; ++i)   // exactly symmetric block
            for (int j = 0; j < i; ++j) w[j][i] = w[i][j];
          const double fo[3] = {f[3 * next], f[3 * next + 1], f[3 * next + 2]};
          double lr[3], dd[3];
          for (int i = 0; i < 3; ++i) lr[i] = F[i][0] * fo[0] + F[i][1] * fo[1] + F[i][2] * fo[2];
          for (int i = 0; i < 3; ++i) dd[i] = delta[i] - (w[i][0] * lr[0] + w[i][1] * lr[1] + w[i][2] * lr[2]);
          double rec[PGS_RW];
          make_record(w, mu[next], rec);
          const Local r = j_inner == 8 ? local_solve_rec<8>(rec, dd, j_inner) : local_solve_rec<0>(rec, dd, j_inner);
          double fn[3], df[3];
          for (int q = 0; q < 3; ++q) {
            fn[q] = F[0][q] * r.l[0] + F[1][q] * r.l[1] + F[2][q] * r.l[2];
            df[q] = fn[q] - fo[q];
            dsum += df[q] * df[q];
          }
          if (ln == 0) {
            for (int q = 0; q < 3; ++q) {
              bc[q] = df[q];
              f[3 * next + q] = fn[q];
              lam[3 * next + q] = r.l[q];
              for (int k = 0; k < 3; ++k) C[9L * next + 3 * q + k] = F[q][k];
            }
            status[next] = (int8_t)r.st;
          }
        }
        if (ln == 0) ctl_s = next;
      }
      __syncthreads();
      const int cur = ctl_s;
      if (cur >= nc) break;
      const double d0 = bc[0], d1 = bc[1], d2 = bc[2];
      if (d0 != 0.0 || d1 != 0.0 || d2 != 0.0) {
        const double *r0 = WH + (3L * cur) * m;
        for (int i = tid; i < m; i += 1024) P[i] += h2 * (r0[i] * d0 + r0[m + i] * d1 + r0[2L * m + i] * d2);
      }
      __syncthreads();
      a = cur + 1;
    }
    // eps = |f_i - f_{i-1}| / |f_i|
    double part = 0.0;
    __threadfence_block();
    for (int i = tid; i < m; i += 1024) part += f[i] * f[i];
    const double nf2 = block_sum(part, red);
    if (tid == 0) {
      const double diff = sqrt(dsum), nf = sqrt(nf2);
      eps = nf > 0.0 ? diff / nf : (diff == 0.0 ? 0.0 : INFINITY);
      stop = (eps <= tol) ? 1 : 0;
    }
    __syncthreads();
    if (stop) {
      ++sweep;
      break;
    }
  }
  if (tid == 0) {
    *sweeps_out = sweep;
    *eps_out = eps;
  }
}

// Active-set projected Gauss-Seidel (exact).  In a sweep only contacts with
// a non-zero force or a negative gap can change; all others are no-ops of
// Gauss-Seidel.  The kernel keeps the set S of contacts that may change and
// runs the sequential sweep over S alone, with the compact coupling block
// W~_SS (gathered once per set) and per-contact records (3x3 block, its
// factor, mu) in LDS.  Up to PGS_WAVE_MAX contacts the sweep is one wave's
// barrier-free chain over register-resident gaps and forces (chain_wave);
// larger sets use a block-wide chain with two barriers per contact.  It
// then verifies that every contact outside S was a no-op at its turn, i.e.
// that its normal gap
//   g_n(c) = g_n^set(c) + W~_{n(c),S} (lambda^turn - lambda^set) >= 0,
// with lambda^turn the force of S contacts before c in this sweep and after c
// from the previous sweep.  Cauchy-Schwarz on the PSD matrix W~ bounds the
// correction by sqrt(W~_cc) * sum_q sqrt(W~_qq) |lambda^turn_q - lambda^set_q|,
// which settles almost every contact; the others are evaluated exactly.  On a
// violation the violating contacts join S and the sweep restarts from its
// start state, so the iterates are those of the full sequential sweep.  If S
// outgrows PGS_SMAX the remaining sweeps go to k_pgs_single (ctl[0] = 1).
constexpr int PGS_SMAX = 512;
constexpr int PGS_S3 = 3 * PGS_SMAX;
constexpr int PGS_NT = 512;   // threads of the active-set kernel
constexpr int PGS_NW = PGS_NT / 64;
constexpr int PGS_WAVE_MAX = kPgsWaveMax;   // largest set swept by the register chains (= PGS_SMAX)
constexpr int PGS_BLK = kPgsBlk;            // doubles per 3x3 block of the blocked W~_SS (9 used, 16-byte aligned)
struct PgsLds {
  double gS[PGS_S3], lamS[PGS_S3], lamS0[PGS_S3], lamSet[PGS_S3];
  double rec[PGS_SMAX * PGS_RW];
  double red[48];
  int Sidx[PGS_SMAX];
  unsigned char stS[PGS_SMAX];
  int wcount[64];
  int ulist[PGS_MAX_NC];
  unsigned char inS[PGS_MAX_NC];
  double Rmin;   // settle threshold of the set: B below it settles every skipped contact
  int nS, flag, stop, nu, zflag, settled;
  int cprog, cflag;   // contacts done by the solving chain; block Gauss-Seidel: next block staged
  int perr;           // a wait of the ring sweep ran out
};

static_assert(sizeof(PgsLds) <= 160 * 1024, "active-set PGS state must fit one CU's LDS");
static_assert(3 * PGS_MAX_NC * sizeof(double) + PGS_MAX_NC + 512 <= 160 * 1024, "k_pgs_single LDS");


__device__ inline double readlane_f64(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Blocks W~(rows of contacts ln + 64k, columns of contact i) for every slot k
// (uniform base, fixed per-lane offset).
template <int NS>
__device__ inline void chain_load(double2 (&X)[NS][PGS_BLK / 2], const double *__restrict__ Wb, int i, int ln) {
  const double2 *base = reinterpret_cast<const double2 *>(Wb + (long)i * (64 * NS * PGS_BLK));
  const int lo = ln * (PGS_BLK / 2);
#pragma unroll
  for (int k = 0; k < NS; ++k)
#pragma unroll
    for (int j = 0; j < PGS_BLK / 2; ++j) X[k][j] = base[lo + k * 64 * (PGS_BLK / 2) + j];
}

// Record and current force of contact i: 11 broadcast 16-byte LDS reads.
struct ChainRec {
  double2 r2[PGS_RW / 2];
  __device__ double operator[](int q) const { return (q & 1) ? r2[q >> 1].y : r2[q >> 1].x; }
};
__device__ inline void chain_rec(ChainRec &c, const PgsLds &L, int i) {
  const double2 *rp = reinterpret_cast<const double2 *>(L.rec + PGS_RW * i);
#pragma unroll
  for (int q = 0; q < PGS_RW / 2; ++q) c.r2[q] = rp[q];
}

// One Gauss-Seidel step of the single-wave chain.  Contact i's gap without
// its own term, e_i = g_i - W~_ii lambda_i (the input of the local solve),
// is in lane i % 64, register slot K = i / 64 (compile-time: no register
// selection); the blocked W~ has zero diagonal blocks, so the update keeps
// e exact.  Every lane runs the local solve on the same broadcast data;
// lane 0 stores the new force and status in LDS; every lane applies
// W~(own rows, i) dlambda_i to its gaps.  Straight-line apart from the local
// solve and the one-lane store, so loads in flight are waited for only where
// they are used.
template <int K, int NS, int J>
__device__ inline void chain_step(int i, const double2 (&X)[NS][PGS_BLK / 2], const ChainRec &c,
                                  double (&g)[NS][3], PgsLds &L, int j_inner, int ln, int o) {
  const int li = i & 63;
  double rc[19];
#pragma unroll
  for (int q = 0; q < 19; ++q) rc[q] = c[q];
  const double lo0 = c[19], lo1 = c[20], lo2 = c[21];
  double dd[3];
  dd[0] = readlane_f64(g[K][0], li);
  dd[1] = readlane_f64(g[K][1], li);
  dd[2] = readlane_f64(g[K][2], li);
  const Local rs = local_solve_rec<J>(rc, dd, j_inner);
  if (ln == 0) {
    double *lp = L.rec + PGS_RW * (i + o) + 19;
    lp[0] = rs.l[0];
    lp[1] = rs.l[1];
    lp[2] = rs.l[2];
    L.stS[i + o] = (unsigned char)rs.st;
  }
  const double d0 = rs.l[0] - lo0, d1 = rs.l[1] - lo1, d2 = rs.l[2] - lo2;
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    const double b[9] = {X[k][0].x, X[k][0].y, X[k][1].x, X[k][1].y, X[k][2].x,
                         X[k][2].y, X[k][3].x, X[k][3].y, X[k][4].x};
#pragma unroll
    for (int a = 0; a < 3; ++a) g[k][a] = fma(b[3 * a + 2], d2, fma(b[3 * a + 1], d1, fma(b[3 * a], d0, g[k][a])));
  }
}

// Contacts 64K .. 64K+63 of the sweep; blocks of the next two contacts and the
// record of the next one are in flight while the current one is solved.
// Loads past the end re-read the last contact (unused).  The set's records,
// statuses and gaps start at contact o of the LDS arrays.  PUB: after every
// two contacts lane 0 publishes how many are done in L.cprog (LDS operations
// of one wave complete in order, so a reader that sees the count sees the
// forces; the compiler fence keeps the stores in that order).
template <int K, int NS, int J, bool PUB>
__device__ inline void chain_slot(int nS, const double *__restrict__ Wb, PgsLds &L, int j_inner, int ln, int o,
                                  double (&g)[NS][3], double2 (&A)[NS][PGS_BLK / 2], double2 (&B)[NS][PGS_BLK / 2],
                                  ChainRec &rA, ChainRec &rB) {
  const int last = nS - 1, end = min(nS, 64 * K + 64);
  for (int i = 64 * K; i < end; i += 2) {
    chain_rec(rB, L, min(i + 1, last) + o);
    chain_step<K, NS, J>(i, A, rA, g, L, j_inner, ln, o);
    chain_load<NS>(A, Wb, min(i + 2, last), ln);
    if (i + 1 < end) {
      chain_rec(rA, L, min(i + 2, last) + o);
      chain_step<K, NS, J>(i + 1, B, rB, g, L, j_inner, ln, o);
    }
    chain_load<NS>(B, Wb, min(i + 3, last), ln);
    if constexpr (PUB) {
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      if (ln == 0) __hip_atomic_store(&L.cprog, min(i + 2, end), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
  }
}

// Sequential sweep over S by wave 0 alone: gaps of S (without own term) live
// in the lanes' registers, forces, records and statuses in LDS; no barrier is
// taken inside the sweep.
template <int NS, int J, bool PUB = false>
__device__ __forceinline__ void chain_wave(int nS, const double *__restrict__ Wb, PgsLds &L, int j_inner,
                                           int o = 0) {
  const int ln = threadIdx.x & 63;
  double g[NS][3];
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    const int c = ln + 64 * k;
#pragma unroll
    for (int q = 0; q < 3; ++q) g[k][q] = c < nS ? L.gS[3 * (c + o) + q] : 0.0;
  }
  const int last = nS - 1;
  double2 A[NS][PGS_BLK / 2], B[NS][PGS_BLK / 2];
  ChainRec rA, rB;
  chain_load<NS>(A, Wb, 0, ln);
  chain_load<NS>(B, Wb, min(1, last), ln);
  chain_rec(rA, L, o);
  chain_slot<0, NS, J, PUB>(nS, Wb, L, j_inner, ln, o, g, A, B, rA, rB);
  if constexpr (NS > 1) chain_slot<1, NS, J, PUB>(nS, Wb, L, j_inner, ln, o, g, A, B, rA, rB);
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    const int c = ln + 64 * k;
    if (c < nS) {
#pragma unroll
      for (int q = 0; q < 3; ++q) L.gS[3 * (c + o) + q] = g[k][q];
    }
  }
}

// Sweep over a set of 65..512 contacts by R = ceil(nS / 64) waves: wave w
// keeps the gaps of contacts 64 w .. 64 w + 63 (one register slot; blocked
// W~_SS columns of nsp contacts).  The contacts are solved in order, each
// 64-contact block by the wave that keeps its gaps, while every other wave
// applies each solved contact's force change to its own gaps as soon as it
// is published; no wave applies another block's updates on the solving
// chain, and no barrier is taken.  The solving wave publishes how many
// contacts are done in L.cprog after the force's stores (LDS operations of
// one wave complete in order); an applying wave takes the change as the
// published force minus the force at the sweep's start (each contact is
// solved once per sweep), so every gap receives the same products in the
// same order as in the one-wave sweep.  A wave solves its block only after
// it has applied every earlier block, so each wait is on a wave that is
// making progress.  A wait that runs out (a broken count, not an input)
// sets L.perr.
// NSP: the padded set size when fixed at compile time (128: two waves), else 0.
constexpr int RING_SPIN = 1 << 24;
template <int NSP>
__device__ inline void ring_load(double2 (&X)[1][PGS_BLK / 2], const double *__restrict__ Wb, int i, int nsp,
                                 int ln, int w) {
  const double2 *base = reinterpret_cast<const double2 *>(Wb + (long)i * (NSP ? NSP : nsp) * PGS_BLK);
  const int lo = (64 * w + ln) * (PGS_BLK / 2);
#pragma unroll
  for (int j = 0; j < PGS_BLK / 2; ++j) X[0][j] = base[lo + j];
}

// The solving part: contacts b .. e-1 (this wave's gaps).
template <int J, int NSP>
__device__ inline void ring_solve(int b, int e, int nsp, const double *__restrict__ Wb, PgsLds &L, int j_inner,
                                  int ln, int w, double (&g)[1][3]) {
  if (b >= e) return;
  const int last = e - 1;
  double2 A[1][PGS_BLK / 2], B[1][PGS_BLK / 2];
  ChainRec rA, rB;
  ring_load<NSP>(A, Wb, b, nsp, ln, w);
  ring_load<NSP>(B, Wb, min(b + 1, last), nsp, ln, w);
  chain_rec(rA, L, b);
  for (int i = b; i < e; i += 2) {
    chain_rec(rB, L, min(i + 1, last));
    chain_step<0, 1, J>(i, A, rA, g, L, j_inner, ln, 0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    if (ln == 0) __hip_atomic_store(&L.cprog, i + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    ring_load<NSP>(A, Wb, min(i + 2, last), nsp, ln, w);
    if (i + 1 < e) {
      chain_rec(rA, L, min(i + 2, last));
      chain_step<0, 1, J>(i + 1, B, rB, g, L, j_inner, ln, 0);
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      if (ln == 0) __hip_atomic_store(&L.cprog, i + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    ring_load<NSP>(B, Wb, min(i + 3, last), nsp, ln, w);
  }
}

// The applying part: the changes of contacts b .. e-1, solved by another
// wave, added to this wave's gaps in contact order.
__device__ inline void ring_apply_one(int i, const double2 (&X)[1][PGS_BLK / 2], PgsLds &L, double (&g)[1][3]) {
  for (int spin = 0; __hip_atomic_load(&L.cprog, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) <= i; ++spin) {
    if (spin == RING_SPIN) {
      __hip_atomic_store(&L.perr, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      break;
    }
    if ((spin & 255) == 255 && __hip_atomic_load(&L.perr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != 0)
      break;   // another wave already gave up: no more waiting in this sweep
    __builtin_amdgcn_s_sleep(1);
  }
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  const double *rp = L.rec + PGS_RW * i + 19;
  const double d0 = rp[0] - L.lamS0[3 * i], d1 = rp[1] - L.lamS0[3 * i + 1], d2 = rp[2] - L.lamS0[3 * i + 2];
  const double bb[9] = {X[0][0].x, X[0][0].y, X[0][1].x, X[0][1].y, X[0][2].x,
                        X[0][2].y, X[0][3].x, X[0][3].y, X[0][4].x};
#pragma unroll
  for (int a = 0; a < 3; ++a) g[0][a] = fma(bb[3 * a + 2], d2, fma(bb[3 * a + 1], d1, fma(bb[3 * a], d0, g[0][a])));
}
template <int NSP>
__device__ inline void ring_apply(int b, int e, int nsp, const double *__restrict__ Wb, PgsLds &L, int ln, int w,
                                  double (&g)[1][3]) {
  if (b >= e) return;
  const int last = e - 1;
  double2 A[1][PGS_BLK / 2], B[1][PGS_BLK / 2];
  ring_load<NSP>(A, Wb, b, nsp, ln, w);
  ring_load<NSP>(B, Wb, min(b + 1, last), nsp, ln, w);
  for (int i = b; i < e; i += 2) {
    ring_apply_one(i, A, L, g);
    ring_load<NSP>(A, Wb, min(i + 2, last), nsp, ln, w);
    if (i + 1 < e) ring_apply_one(i + 1, B, L, g);
    ring_load<NSP>(B, Wb, min(i + 3, last), nsp, ln, w);
  }
}

template <int J, int NSP>
__device__ __forceinline__ void chain_ring(int nS, int nsp, const double *__restrict__ Wb, PgsLds &L, int j_inner,
                                           int w) {
  const int ln = threadIdx.x & 63, c = 64 * w + ln, R = (nS + 63) / 64;
  double g[1][3];
#pragma unroll
  for (int q = 0; q < 3; ++q) g[0][q] = c < nS ? L.gS[3 * c + q] : 0.0;
  if constexpr (NSP == 128) {   // two waves: one block each
    const int h = min(64, nS);
    if (w == 0) {
      ring_solve<J, NSP>(0, h, nsp, Wb, L, j_inner, ln, w, g);
      ring_apply<NSP>(h, nS, nsp, Wb, L, ln, w, g);
    } else {
      ring_apply<NSP>(0, h, nsp, Wb, L, ln, w, g);
      ring_solve<J, NSP>(h, nS, nsp, Wb, L, j_inner, ln, w, g);
    }
  } else {
    for (int b = 0; b < R; ++b) {
      const int lo = 64 * b, hi = min(lo + 64, nS);
      if (b == w)
        ring_solve<J, NSP>(lo, hi, nsp, Wb, L, j_inner, ln, w, g);
      else
        ring_apply<NSP>(lo, hi, nsp, Wb, L, ln, w, g);
    }
  }
  if (c < nS) {
#pragma unroll
    for (int q = 0; q < 3; ++q) L.gS[3 * c + q] = g[0][q];
  }
}

// The active set of the first sweep, its compact couplings and records are
// prepared by a wide kernel before the sequential kernel starts (a set that
// grows later is rebuilt inside k_pgs_active).
// k_pgs_gather (any grid): the normal gaps at the set's start and sqrt(W~_nn)
// of every contact; every block forms the set S = {c : lambda_c != 0 or
// g0_n(c) < 0} in ascending order (64-contact ballots, window prefix) and
// block 0 writes S and |S|.  For a set of at most PGS_WAVE_MAX contacts the blocks then
// write the blocked W~_SS with zero diagonal blocks, the per-contact records
// and the gaps without the own term, e = g0 - W~_cc lambda_c.
template <class TW>
__global__ __launch_bounds__(256) void k_pgs_gather(int nc, const TW *__restrict__ W,
                                                    const double *__restrict__ g0, const double *__restrict__ lam,
                                                    const double *__restrict__ mu, double h2,
                                                    int *__restrict__ Sidx_out, int *__restrict__ nS_out,
                                                    double *__restrict__ gnSet, double *__restrict__ swn,
                                                    double *__restrict__ Wss, double *__restrict__ rec,
                                                    double *__restrict__ gS) {
  __shared__ int Sidx[PGS_MAX_NC];
  __shared__ int wcount[PGS_MAX_NC / 64 + 1];
  __shared__ int nS_s;
  const int m = 3 * nc;
  const int tid = threadIdx.x, wv = tid >> 6, ln = tid & 63;
  const int nwin = (nc + 63) / 64;
  const long stride = (long)gridDim.x * blockDim.x, t0 = (long)blockIdx.x * blockDim.x + threadIdx.x;
  for (long c = t0; c < nc; c += stride) {
    gnSet[c] = g0[3 * c];
    swn[c] = sqrt(h2 * (double)W[(3L * c) * m + 3L * c]);
  }
  auto in_set = [&](int c) {
    return c < nc && (lam[3 * c] != 0.0 || lam[3 * c + 1] != 0.0 || lam[3 * c + 2] != 0.0 || g0[3 * c] < 0.0);
  };
  for (int w = wv; w < nwin; w += 4) {
    const unsigned long long bal = __ballot(in_set(64 * w + ln));
    if (ln == 0) wcount[w] = __popcll(bal);
  }
  __syncthreads();
  if (tid == 0) {
    int acc = 0;
    for (int w = 0; w < nwin; ++w) {
      const int t = wcount[w];
      wcount[w] = acc;
      acc += t;
    }
    nS_s = acc;
  }
  __syncthreads();
  for (int w = wv; w < nwin; w += 4) {
    const int c = 64 * w + ln;
    const bool in = in_set(c);
    const unsigned long long bal = __ballot(in);
    if (in) Sidx[wcount[w] + __popcll(bal & ((1ull << ln) - 1ull))] = c;
  }
  __syncthreads();
  const int nS = nS_s;
  if (blockIdx.x == 0) {
    for (int q = tid; q < nS; q += 256) Sidx_out[q] = Sidx[q];
    if (tid == 0) *nS_out = nS;
  }
  if (nS == 0 || nS > PGS_WAVE_MAX) return;
  const int nsp = pgs_wave_pad(nS);
  const long nel = (long)nS * nsp * PGS_BLK;
  for (long e = t0; e < nel; e += stride) {
    const int j = (int)(e % PGS_BLK);
    const long ic = e / PGS_BLK;
    const int c = (int)(ic % nsp), i = (int)(ic / nsp);
    double v = 0.0;
    if (j < 9 && c < nS && c != i) v = h2 * (double)W[(3L * Sidx[c] + j / 3) * m + 3L * Sidx[i] + j % 3];
    Wss[e] = v;
  }
  for (long i = t0; i < nS; i += stride) {
    double wb[3][3];
    const long ci = 3L * Sidx[i];
    for (int p = 0; p < 3; ++p)
      for (int q = 0; q < 3; ++q) wb[p][q] = h2 * (double)W[(ci + p) * m + ci + q];
    double tmp[19];
    make_record(wb, mu[Sidx[i]], tmp);
    for (int q = 0; q < 19; ++q) rec[PGS_RW * i + q] = tmp[q];
  }
  for (long r = t0; r < 3L * nS; r += stride) {
    const long cr = 3L * Sidx[r / 3];
    const int a = (int)(r % 3);
    double own = 0.0;
    for (int q = 0; q < 3; ++q) own = fma(h2 * (double)W[(cr + a) * m + cr + q], lam[cr + q], own);
    gS[r] = g0[cr + a] - own;
  }
}

// The sequential kernel's body, for one workgroup of PGS_NT threads with the
// state L in its LDS (k_pgs_active, and each scene's workgroup of the batched
// Newton loop).  npre: size of the set prepared by k_pgs_gather (preSidx,
// preRec, preGS); a value above PGS_WAVE_MAX builds the first set here, from
// g0, gnSet and swn.
template <class TW>
__device__ __forceinline__ void pgs_active_body(PgsLds &L, int nc, const TW *__restrict__ W,
                                                const double *__restrict__ d, const double *__restrict__ g0,
                                                const double *__restrict__ mu, double h2, double *__restrict__ lam,
                                                int8_t *__restrict__ status, int max_sweeps, double tol,
                                                int j_inner, int *__restrict__ sweeps_out,
                                                double *__restrict__ eps_out, double *__restrict__ Wss,
                                                double *__restrict__ gnSet, const double *__restrict__ swn,
                                                int *__restrict__ ctl, const int *__restrict__ preSidx, int npre,
                                                const double *__restrict__ preRec, const double *__restrict__ preGS) {
  const int m = 3 * nc;
  const int tid = threadIdx.x, wv = tid >> 6, ln = tid & 63;
  for (int c = tid; c < nc; c += PGS_NT) {
    bool nzc = lam[3 * c] != 0.0 || lam[3 * c + 1] != 0.0 || lam[3 * c + 2] != 0.0;
    L.inS[c] = (nzc || g0[3 * c] < 0.0) ? 1 : 0;
  }
  if (tid == 0) {
    L.stop = 0;
    L.zflag = 0;
    L.perr = 0;
    ctl[0] = 0;
    ctl[1] = 0;
  }
  __syncthreads();
  int sweep = 0, nS = 0, ldS = 0, nsp = 0;
  double eps = 0.0;
  bool need_build = true, first_build = true, built = false;
  while (sweep < max_sweeps) {
    if (need_build && first_build && npre <= PGS_WAVE_MAX) {
      // ---- the prepared first set: copy it in
      nS = npre;
      ldS = 3 * nS;
      nsp = pgs_wave_pad(nS);
      for (int i = tid; i < nS; i += PGS_NT) L.Sidx[i] = preSidx[i];
      for (int e = tid; e < nS * 19; e += PGS_NT) L.rec[PGS_RW * (e / 19) + e % 19] = preRec[PGS_RW * (e / 19) + e % 19];
      for (int r = tid; r < ldS; r += PGS_NT) L.gS[r] = preGS[r];
      __syncthreads();
      for (int r = tid; r < ldS; r += PGS_NT) {
        L.lamS[r] = lam[3 * L.Sidx[r / 3] + r % 3];
        L.lamSet[r] = L.lamS[r];
      }
      __syncthreads();
      need_build = false;
      first_build = false;
      built = true;
    }
    if (need_build) {
      // ---- ordered list of S (ballot per 64-contact window, prefix by thread 0)
      const int nwin = (nc + 63) / 64;
      for (int w = wv; w < nwin; w += PGS_NW) {
        const int c = 64 * w + ln;
        const unsigned long long bal = __ballot(c < nc && L.inS[c]);
        if (ln == 0) L.wcount[w] = __popcll(bal);
      }
      __syncthreads();
      if (tid == 0) {
        int acc = 0;
        for (int w = 0; w < nwin; ++w) {
          int t = L.wcount[w];
          L.wcount[w] = acc;
          acc += t;
        }
        L.nS = acc;
      }
      __syncthreads();
      nS = L.nS;
      if (nS > PGS_SMAX) {   // hand over: global lambda holds the sweep-start state
        if (tid == 0) {
          ctl[0] = 1;
          ctl[1] = sweep;
        }
        return;
      }
      for (int w = wv; w < nwin; w += PGS_NW) {
        const int c = 64 * w + ln;
        const bool in = c < nc && L.inS[c];
        const unsigned long long bal = __ballot(in);
        if (in) L.Sidx[L.wcount[w] + __popcll(bal & ((1ull << ln) - 1ull))] = c;
      }
      __syncthreads();
      ldS = 3 * nS;
      nsp = pgs_wave_pad(nS);
      for (int r = tid; r < ldS; r += PGS_NT) {
        L.lamS[r] = lam[3 * L.Sidx[r / 3] + r % 3];
        L.lamSet[r] = L.lamS[r];
      }
      // ---- compact couplings W~_SS: blocked [i][c] 3x3 blocks of rows c,
      // columns i (padded to nsp contacts), zero diagonal blocks
      {
        const long nel = (long)nS * nsp * PGS_BLK;
        for (long e = tid; e < nel; e += PGS_NT) {
          const int j = (int)(e % PGS_BLK);
          const long ic = e / PGS_BLK;
          const int c = (int)(ic % nsp), i = (int)(ic / nsp);
          double v = 0.0;
          if (j < 9 && c < nS && c != i) v = h2 * (double)W[(3L * L.Sidx[c] + j / 3) * m + 3L * L.Sidx[i] + j % 3];
          Wss[e] = v;
        }
      }
      __threadfence_block();
      __syncthreads();
      for (int i = tid; i < nS; i += PGS_NT) {
        double wb[3][3];
        const long ci = 3L * L.Sidx[i];
        for (int p = 0; p < 3; ++p)
          for (int q = 0; q < 3; ++q) wb[p][q] = h2 * (double)W[(ci + p) * m + ci + q];
        double *rc = L.rec + PGS_RW * i;
        double tmp[19];
        make_record(wb, mu[L.Sidx[i]], tmp);
        for (int q = 0; q < 19; ++q) rc[q] = tmp[q];
      }
      // ---- gaps at the set's start state (lambda is zero outside S)
      if (first_build) {
        // g0 = d + W~ lambda0 was formed by k_sym_gemv_sparse for every row; the
        // chains keep the gap without the contact's own term
        for (int r = tid; r < ldS; r += PGS_NT) {
          const long cr = 3L * L.Sidx[r / 3];
          double own = 0.0;
          for (int q = 0; q < 3; ++q) own = fma(h2 * (double)W[(cr + r % 3) * m + cr + q], L.lamS[r - r % 3 + q], own);
          L.gS[r] = g0[cr + r % 3] - own;
        }
      } else {
        for (int c = wv; c < nS; c += PGS_NW) {
          double a0 = 0.0, a1 = 0.0, a2 = 0.0;
          for (int i = ln; i < nS; i += 64) {
            const double *b = Wss + ((long)i * nsp + c) * PGS_BLK;
            const double l0 = L.lamS[3 * i], l1 = L.lamS[3 * i + 1], l2 = L.lamS[3 * i + 2];
            a0 += b[0] * l0 + b[1] * l1 + b[2] * l2;
            a1 += b[3] * l0 + b[4] * l1 + b[5] * l2;
            a2 += b[6] * l0 + b[7] * l1 + b[8] * l2;
          }
          for (int o = 32; o > 0; o >>= 1) {
            a0 += __shfl_xor(a0, o, 64);
            a1 += __shfl_xor(a1, o, 64);
            a2 += __shfl_xor(a2, o, 64);
          }
          if (ln == 0) {
            const int cc = 3 * L.Sidx[c];
            L.gS[3 * c] = d[cc] + a0;
            L.gS[3 * c + 1] = d[cc + 1] + a1;
            L.gS[3 * c + 2] = d[cc + 2] + a2;
          }
        }
        for (int c = wv; c < nc; c += PGS_NW) {
          if (L.inS[c]) continue;
          double a = 0.0;
          for (int q = ln; q < ldS; q += 64)
            a = fma(h2 * (double)W[(3L * c) * m + 3L * L.Sidx[q / 3] + q % 3], L.lamS[q], a);
          for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
          if (ln == 0) gnSet[c] = d[3 * c] + a;
        }
      }
      __syncthreads();
      need_build = false;
      first_build = false;
      built = true;
    }
    if (built) {
      // Settle threshold of the new set.  A skipped contact c is settled when
      // g - sqrt(W~_cc) B > 1e-13 (|g| + sqrt(W~_cc) B), i.e. (sqrt(W~_cc) > 0)
      // B < (g - 1e-13 |g|) / (sqrt(W~_cc) (1 + 1e-13)); Rmin is the smallest
      // of these bounds, shrunk by 1e-12 for rounding, so B < Rmin settles
      // all of them at once (else the per-contact test runs).
      double rmin = INFINITY;
      int zf = 0;
      for (int c = tid; c < nc; c += PGS_NT) {
        if (L.inS[c]) continue;
        const double g = gnSet[c], w = swn[c];
        if (w > 0.0)
          rmin = fmin(rmin, (g - 1e-13 * fabs(g)) / (w * (1.0 + 1e-13)));
        else if (!(g > 0.0))
          zf = 1;
        status[c] = (int8_t)ICR_SEPARATE;
      }
      if (zf) atomicOr(&L.zflag, 1);
      const double rm = block_min(rmin, L.red);
      if (tid == 0) L.Rmin = rm > 0.0 ? rm * (1.0 - 1e-12) : rm * (1.0 + 1e-12);
      __syncthreads();
      built = false;
    }
    // ---- sweep over S from its start state (forces into the records)
    for (int r = tid; r < ldS; r += PGS_NT) {
      L.lamS0[r] = L.lamS[r];
      L.rec[PGS_RW * (r / 3) + 19 + r % 3] = L.lamS[r];
    }
    if (tid == 0) {
      L.flag = 0;
      L.nu = 0;
      L.cprog = 0;
    }
    __syncthreads();
    if (nS > 0) {
      if (nS <= 64) {
        if (wv == 0) {
          if (j_inner == 8)
            chain_wave<1, 8>(nS, Wss, L, j_inner);
          else
            chain_wave<1, 0>(nS, Wss, L, j_inner);
        }
      } else if (nS <= 128) {
        if (wv < 2) {
          if (j_inner == 8)
            chain_ring<8, 128>(nS, nsp, Wss, L, j_inner, wv);
          else
            chain_ring<0, 128>(nS, nsp, Wss, L, j_inner, wv);
        }
      } else if (wv < (nS + 63) / 64) {
        if (j_inner == 8)
          chain_ring<8, 0>(nS, nsp, Wss, L, j_inner, wv);
        else
          chain_ring<0, 0>(nS, nsp, Wss, L, j_inner, wv);
      }
    }
    __syncthreads();
    // ---- one pass over S: sum of squared changes of the sweep, |lambda|^2,
    // and the bound factor of the skipped contacts' gaps
    // B = sum_q sqrt(W~_qq) max(|lamS - lamSet|, |lamS0 - lamSet|)
    // (the forces come back from the records in the same pass)
    double dpart = 0.0, bpart = 0.0, npart = 0.0;
    for (int r = tid; r < ldS; r += PGS_NT) {
      const double *rc = L.rec + PGS_RW * (r / 3);
      const double wqq = (r % 3 == 0) ? rc[0] : ((r % 3 == 1) ? rc[3] : rc[5]);
      const double ls = rc[19 + r % 3], l0 = L.lamS0[r], lset = L.lamSet[r];
      L.lamS[r] = ls;
      const double dv = ls - l0;
      dpart += dv * dv;
      bpart += sqrt(wqq) * fmax(fabs(ls - lset), fabs(l0 - lset));
      npart += ls * ls;
    }
    block_sum3(dpart, bpart, npart, L.red);
    if (tid == 0) {
      const double diff = sqrt(dpart), nl = sqrt(npart);
      eps = nl > 0.0 ? diff / nl : (diff == 0.0 ? 0.0 : INFINITY);
      if (L.perr) eps = NAN;   // the ring sweep lost its count: stop and report eps = NaN
      L.stop = (eps <= tol || L.perr) ? 1 : 0;
      L.red[0] = bpart * (1.0 + 1e-12);
      L.settled = (L.zflag == 0 && L.red[0] < L.Rmin) ? 1 : 0;
    }
    __syncthreads();
    const double B = L.red[0];
    // ---- verify the skipped contacts (all settled at once when B < Rmin)
    if (!L.settled) {
      for (int c = tid; c < nc; c += PGS_NT) {
        if (L.inS[c]) continue;
        const double g = gnSet[c], rb = swn[c] * B;
        if (!(g - rb > 1e-13 * (fabs(g) + rb))) L.ulist[atomicAdd(&L.nu, 1)] = c;
      }
      __syncthreads();
      const int nu = L.nu;
      for (int u = wv; u < nu; u += PGS_NW) {   // exact gap at the turn of the unsettled contacts
        const int c = L.ulist[u];
        double a = 0.0;
        for (int q = ln; q < ldS; q += 64) {
          const double lt = (L.Sidx[q / 3] < c) ? L.lamS[q] : L.lamS0[q];
          a = fma(h2 * (double)W[(3L * c) * m + 3L * L.Sidx[q / 3] + q % 3], lt - L.lamSet[q], a);
        }
        for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
        if (ln == 0 && gnSet[c] + a < 0.0) {
          L.inS[c] = 1;
          L.flag = 1;
        }
      }
      __syncthreads();
    }
    if (L.flag && !L.perr) {
      // a skipped contact was not a no-op: restart the sweep with a larger S
      for (int r = tid; r < ldS; r += PGS_NT) lam[3 * L.Sidx[r / 3] + r % 3] = L.lamS0[r];
      need_build = true;
      __threadfence_block();
      __syncthreads();
      continue;
    }
    ++sweep;
    if (L.stop) break;
  }
  for (int r = tid; r < ldS; r += PGS_NT) lam[3 * L.Sidx[r / 3] + r % 3] = L.lamS[r];
  for (int i = tid; i < nS; i += PGS_NT) status[L.Sidx[i]] = (int8_t)L.stS[i];
  if (tid == 0) {
    *sweeps_out = sweep;
    *eps_out = eps;
  }
}

template <class TW>
__global__ __launch_bounds__(PGS_NT) void k_pgs_active(int nc, const TW *__restrict__ W,
                                                       const double *__restrict__ d, const double *__restrict__ g0,
                                                       const double *__restrict__ mu, double h2,
                                                       double *__restrict__ lam, int8_t *__restrict__ status,
                                                       int max_sweeps, double tol, int j_inner,
                                                       int *__restrict__ sweeps_out, double *__restrict__ eps_out,
                                                       double *__restrict__ Wss, double *__restrict__ gnSet,
                                                       const double *__restrict__ swn, int *__restrict__ ctl,
                                                       const int *__restrict__ preSidx, const int *__restrict__ preN,
                                                       const double *__restrict__ preRec,
                                                       const double *__restrict__ preGS) {
  extern __shared__ double lds_raw[];
  PgsLds &L = *reinterpret_cast<PgsLds *>(lds_raw);
  pgs_active_body<TW>(L, nc, W, d, g0, mu, h2, lam, status, max_sweeps, tol, j_inner, sweeps_out, eps_out, Wss,
                      gnSet, swn, ctl, preSidx, *preN, preRec, preGS);
}

// ---- batched Newton loops: one workgroup per scene --------------------------
//
// y[i] = x0[i] + h2 sum over the contacts c with a non-zero block of v
// (ascending) of M[(3c + a) m + i] v[3c + a], by one workgroup (M symmetric,
// rows of M read for its columns).  The order of every sum is that of
// k_sym_gemv_sparse (one 64-row block at a time, wave w takes list entries
// w, w + 8, ..., the eight partial sums added in wave order), so the result
// is bit-for-bit the per-scene kernel's.  The contacts taken are those with
// a non-zero block of nzv (the forces lambda, also when v is f = C^T lambda,
// as there); list (LDS) receives them, part (LDS) holds 8 x 64 partial sums.
template <class TM>
__device__ void wg_sym_gemv_sparse(int nc, const TM *__restrict__ M, const double *__restrict__ x0,
                                   const double *__restrict__ v, const double *__restrict__ nzv, double h2,
                                   double *__restrict__ y, int *list, int *count, double *part) {
  static_assert(PGS_NT == SG_NT, "the per-scene kernel's wave count");
  const int tid = threadIdx.x, wv = tid >> 6, ln = tid & 63;
  const long m = 3L * nc;
  if (wv == 0) {
    int cnt = 0;
    for (int c0 = 0; c0 < nc; c0 += 64) {
      const int c = c0 + ln;
      const bool nz = c < nc && block_nonzero(nzv, c);
      const unsigned long long bal = __ballot(nz);
      if (nz) list[cnt + __popcll(bal & ((1ull << ln) - 1ull))] = c;
      cnt += __popcll(bal);
    }
    if (ln == 0) *count = cnt;
  }
  __syncthreads();
  const int n = *count;
  for (long i0 = 0; i0 < m; i0 += 64) {
    const long i = i0 + ln;
    double s = 0.0;
    if (i < m) {
#pragma unroll 4
      for (int q = wv; q < n; q += SG_NW) {
        const long r = 3L * list[q];
        s = fma((double)M[r * m + i], v[r], s);
        s = fma((double)M[(r + 1) * m + i], v[r + 1], s);
        s = fma((double)M[(r + 2) * m + i], v[r + 2], s);
      }
    }
    part[wv * 64 + ln] = s;
    __syncthreads();
    if (wv == 0 && i < m) {
      double t = 0.0;
      for (int w = 0; w < SG_NW; ++w) t += part[w * 64 + ln];
      y[i] = x0[i] + h2 * t;
    }
    __syncthreads();
  }
}

// Algorithm 3's Newton loop (steps 1-4) of one scene per workgroup: frames
// and gaps at the last proximity (the warm start in the new frames), W_k =
// C_k W_H C_k^T, the PGS start gaps g0 = d + W~ lambda, the active-set PGS
// (the sequential kernel's body; the first set is built in place), and the
// world forces f = C^T lambda with the proximity p = p_free + h^2 W_H f
// (Eq. 31).  Every value is computed as the per-scene kernels compute it, in
// the same order, so a step's results do not depend on the path it took.
// The task table as the device reads it: the same layout with every pointer
// in the global address space, so that the code inlined below uses global
// loads and their counters (a pointer read from memory is otherwise generic).
template <class T>
using gptr = __attribute__((address_space(1))) T *;
struct NewtonTaskG {
  int nc, n_newton, max_sweeps, j_inner;
  double tol, h;
  gptr<const StepCtx> ctx;
  gptr<const double> WH, pfree, pstart, mu;
  gptr<double> W, p, f, C, dk, lam, eps;
  gptr<double> g, Wss, gnSet, swn;
  gptr<int8_t> status;
  gptr<int> sweeps, ctl;
};
static_assert(sizeof(NewtonTaskG) == sizeof(NewtonTask) && offsetof(NewtonTaskG, ctl) == offsetof(NewtonTask, ctl),
              "device view of the task table");

__global__ __launch_bounds__(PGS_NT) void k_newton_batch(const NewtonTask *__restrict__ tasks, NewtonBatchIdx ids) {
  extern __shared__ double lds_raw[];
  PgsLds &L = *reinterpret_cast<PgsLds *>(lds_raw);
  const NewtonTaskG &tg = reinterpret_cast<const NewtonTaskG *>(tasks)[ids.idx[blockIdx.x]];
  struct {
    int nc, n_newton, max_sweeps, j_inner;
    double tol, h;
    const StepCtx *ctx;
    const double *WH, *pfree, *pstart, *mu;
    double *W, *p, *f, *C, *dk, *lam, *eps;
    int8_t *status;
    int *sweeps;
  } t{tg.nc, tg.n_newton, tg.max_sweeps, tg.j_inner, tg.tol, tg.h, (const StepCtx *)tg.ctx,
      (const double *)tg.WH, (const double *)tg.pfree, (const double *)tg.pstart, (const double *)tg.mu,
      (double *)tg.W, (double *)tg.p, (double *)tg.f, (double *)tg.C, (double *)tg.dk, (double *)tg.lam,
      (double *)tg.eps, (int8_t *)tg.status, (int *)tg.sweeps};
  struct {
    double *g, *Wss, *gnSet, *swn;
    int *ctl;
  } w{(double *)tg.g, (double *)tg.Wss, (double *)tg.gnSet, (double *)tg.swn, (int *)tg.ctl};
  const int nc = t.nc, tid = threadIdx.x;
  const long m = 3L * nc;
  const double h2 = t.h * t.h;
  for (int k = 0; k < t.n_newton; ++k) {
    // step 1: frames and gaps at p_{k-1} (p_free for the first iteration)
    {
      const icr_obstacle obs = t.ctx->obs;
      const double t0 = t.ctx->t0, t1 = t.ctx->t0 + t.ctx->h;
      const double *p = (k == 0) ? t.pfree : t.p;
      for (int c = tid; c < nc; c += PGS_NT) {
        double pc[3] = {p[3 * c], p[3 * c + 1], p[3 * c + 2]};
        double ps[3] = {t.pstart[3 * c], t.pstart[3 * c + 1], t.pstart[3 * c + 2]};
        double F[3][3], delta[3];
        contact_frame(obs, t0, t1, pc, ps, F, delta);
        double dp[3] = {pc[0] - t.pfree[3 * c], pc[1] - t.pfree[3 * c + 1], pc[2] - t.pfree[3 * c + 2]};
        for (int r = 0; r < 3; ++r) {
          for (int a = 0; a < 3; ++a) t.C[9 * c + 3 * r + a] = F[r][a];
          t.dk[3 * c + r] = delta[r] - (F[r][0] * dp[0] + F[r][1] * dp[1] + F[r][2] * dp[2]);
          t.lam[3 * c + r] = F[r][0] * t.f[3 * c] + F[r][1] * t.f[3 * c + 1] + F[r][2] * t.f[3 * c + 2];
        }
      }
    }
    __syncthreads();
    // step 2: W_k = C_k W_H C_k^T
    for (long blk = tid; blk < (long)nc * nc; blk += PGS_NT) update_W_block(nc, t.WH, t.C, t.W, blk);
    __syncthreads();
    // PGS start gaps and the per-contact set data
    wg_sym_gemv_sparse<double>(nc, t.W, t.dk, t.lam, t.lam, h2, w.g, L.ulist, &L.nu, L.lamS);
    for (int c = tid; c < nc; c += PGS_NT) {
      w.gnSet[c] = w.g[3 * c];
      w.swn[c] = sqrt(h2 * t.W[(3L * c) * m + 3L * c]);
    }
    __syncthreads();
    // step 3: PGS
    pgs_active_body<double>(L, nc, t.W, t.dk, w.g, t.mu, h2, t.lam, t.status, t.max_sweeps, t.tol, t.j_inner,
                            t.sweeps + k, t.eps + k, w.Wss, w.gnSet, w.swn, w.ctl, nullptr, PGS_WAVE_MAX + 1,
                            nullptr, nullptr);
    __syncthreads();
    // step 4: world forces and the proximity update (Eq. 31)
    for (long e = tid; e < m; e += PGS_NT) t.f[e] = world_force(t.C, t.lam, e / 3, (int)(e % 3));
    __syncthreads();
    wg_sym_gemv_sparse<double>(nc, t.WH, t.pfree, t.f, t.lam, h2, t.p, L.ulist, &L.nu, L.lamS);
  }
}

// ---- directions updated before every local solve, on the register chain ----
//
// The per-constraint Gauss-Seidel (R18, k_pgs_pc) with the structure of
// k_pgs_active: only contacts with a force or a negative normal gap can
// change (a contact with no force whose gap at its turn is >= 0 stays
// separated: a no-op), so the sweep runs over the set S of those contacts
// alone.  Wave 0 holds their proximities P (world frame) in registers; at
// contact a's turn it takes its frame and gap at P_a, the block
// W~_aa = h^2 C_a W_H,aa C_a^T, the gap without the own force, the local
// solve and f_a = C_a^T lambda_a with the same arithmetic as k_pgs_pc, then
// every lane adds h^2 W_H(own rows, a) (f_a - f_a^old) to its proximities.
// After a sweep every contact c outside S is verified to have been a no-op:
// its proximity at its turn is P_c^set + h^2 sum_{b in S} W_H,cb
// (f_b^turn - f_b^set) (forces of S contacts before c in this sweep, after
// it from the previous sweep); the signed distance is 1-Lipschitz and
// |h^2 W_H,cb| <= h sqrt(tr W_H,cc) h sqrt(tr W_H,bb) for the PSD W_H, so
// phi_set(c) > h sqrt(tr W_H,cc) B with
// B = sum_b h sqrt(tr W_H,bb) max(|f_b^new - f_b^set|, |f_b^old - f_b^set|)
// settles c, and the others get their exact proximity and gap.  A violation
// adds the contact to S and restarts the sweep from its start state; a set
// beyond 128 contacts hands over to k_pgs_pc (ctl[0] = 1, the sweep in
// ctl[1], the proximity of the hand-over state in Pset).
constexpr int PCA_MAX = 128;   // contacts of S in the single-wave chain
constexpr int PCA_RW = 26;     // record of a contact of S, see PcaLds
struct PcaLds {
  double P[3 * PCA_MAX];       // proximity of S (the chain's registers between sweeps)
  // per contact of S: 0-5 W_H,aa (w00 w01 w02 w11 w12 w22), 6 mu, 7-9 p_start,
  // 10-12 lambda, 13-21 frame rows, 22-24 world force f, 25 unused
  double rec[PCA_MAX * PCA_RW];
  double f0[3 * PCA_MAX];      // forces of S at the sweep's start
  double fset[3 * PCA_MAX];    // ... at the set's start state
  double part[8 * 64];         // partial sums of the proximity product
  double red[48];
  int Sidx[PCA_MAX];
  unsigned char stS[PCA_MAX];
  int wcount[64];
  int ulist[PGS_MAX_NC];
  unsigned char inS[PGS_MAX_NC];
  int nS, flag, stop, nu;
  int cprog, perr;   // two-wave sweep: contacts done by the solving wave; a wait ran out
};
static_assert(sizeof(PcaLds) <= 160 * 1024, "per-constraint chain state must fit one CU's LDS");

struct PcaRec {
  double2 r2[PCA_RW / 2];
  __device__ double operator[](int q) const { return (q & 1) ? r2[q >> 1].y : r2[q >> 1].x; }
};
__device__ inline void pca_rec(PcaRec &c, const PcaLds &L, int i) {
  const double2 *rp = reinterpret_cast<const double2 *>(L.rec + PCA_RW * i);
#pragma unroll
  for (int q = 0; q < PCA_RW / 2; ++q) c.r2[q] = rp[q];
}

// contact_frame with each normalisation by the refined reciprocal square
// root of the squared length (the length itself is that square times it):
// within an ulp or two of the square roots and divisions, and a short
// dependent chain; the frame of every visit of the chain.
__device__ inline void contact_frame_rcp(const icr_obstacle &obs, double t0, double t1, const double pc[3],
                                         const double ps[3], double F[3][3], double delta[3]) {
  double n[3], phi;
  {
#pragma clang fp contract(off)
    const double c[3] = {obs.c0[0] + obs.vel[0] * t1, obs.c0[1] + obs.vel[1] * t1, obs.c0[2] + obs.vel[2] * t1};
    const double r0 = pc[0] - c[0], r1 = pc[1] - c[1], r2 = pc[2] - c[2];
    if (obs.kind == 1) {
      const double d2 = r0 * r0 + r1 * r1 + r2 * r2;
      const double id = frsqrt(d2);
      n[0] = r0 * id;
      n[1] = r1 * id;
      n[2] = r2 * id;
      phi = d2 * id - obs.radius;
    } else {
      n[0] = obs.normal[0];
      n[1] = obs.normal[1];
      n[2] = obs.normal[2];
      phi = r0 * obs.normal[0] + r1 * obs.normal[1] + r2 * obs.normal[2];
    }
  }
  int ax = 0;
  double am = fabs(n[0]);
  if (fabs(n[1]) < am) {
    ax = 1;
    am = fabs(n[1]);
  }
  if (fabs(n[2]) < am) ax = 2;
  const double en = n[ax];
  double ta[3] = {-en * n[0], -en * n[1], -en * n[2]};
  ta[ax] += 1.0;
  const double itn = frsqrt(ta[0] * ta[0] + ta[1] * ta[1] + ta[2] * ta[2]);
  ta[0] *= itn;
  ta[1] *= itn;
  ta[2] *= itn;
  const double tb[3] = {n[1] * ta[2] - n[2] * ta[1], n[2] * ta[0] - n[0] * ta[2], n[0] * ta[1] - n[1] * ta[0]};
  double rel[3];
  for (int a = 0; a < 3; ++a) {
    const double uo = (obs.c0[a] + obs.vel[a] * t1) - (obs.c0[a] + obs.vel[a] * t0);
    rel[a] = pc[a] - ps[a] - uo;
  }
  for (int a = 0; a < 3; ++a) {
    F[0][a] = n[a];
    F[1][a] = ta[a];
    F[2][a] = tb[a];
  }
  delta[0] = phi;
  delta[1] = ta[0] * rel[0] + ta[1] * rel[1] + ta[2] * rel[2];
  delta[2] = tb[0] * rel[0] + tb[1] * rel[1] + tb[2] * rel[2];
}

// One visit of the chain: contact i, its proximity in lane i % 64, slot K.
template <int K, int NS, int J>
__device__ inline void pca_step(int i, const double2 (&X)[NS][PGS_BLK / 2], const PcaRec &c, double (&g)[NS][3],
                                PcaLds &L, int j_inner, int ln, const icr_obstacle &obs, double t0, double t1,
                                double h2) {
  const int li = i & 63;
  const double pa[3] = {readlane_f64(g[K][0], li), readlane_f64(g[K][1], li), readlane_f64(g[K][2], li)};
  const double ps[3] = {c[7], c[8], c[9]};
  double F[3][3], delta[3];
  contact_frame_rcp(obs, t0, t1, pa, ps, F, delta);
  const double wh[3][3] = {{c[0], c[1], c[2]}, {c[1], c[3], c[4]}, {c[2], c[4], c[5]}};
  double B[3][3];   // W_H,aa C_a^T
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) B[a][b] = wh[a][0] * F[b][0] + wh[a][1] * F[b][1] + wh[a][2] * F[b][2];
  double w[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) w[a][b] = h2 * (F[a][0] * B[0][b] + F[a][1] * B[1][b] + F[a][2] * B[2][b]);
  for (int a = 0; a < 3; ++a)   // exactly symmetric block
    for (int b = 0; b < a; ++b) w[b][a] = w[a][b];
  const double fo[3] = {c[22], c[23], c[24]};
  double lr[3], dd[3];
  for (int a = 0; a < 3; ++a) lr[a] = F[a][0] * fo[0] + F[a][1] * fo[1] + F[a][2] * fo[2];
  for (int a = 0; a < 3; ++a) dd[a] = delta[a] - (w[a][0] * lr[0] + w[a][1] * lr[1] + w[a][2] * lr[2]);
  double rc[PGS_RW];
  make_record<true>(w, c[6], rc);
  const Local r = local_solve_rec<J>(rc, dd, j_inner);
  double fn[3], df[3];
  for (int q = 0; q < 3; ++q) {
    fn[q] = F[0][q] * r.l[0] + F[1][q] * r.l[1] + F[2][q] * r.l[2];
    df[q] = fn[q] - fo[q];
  }
  if (ln == 0) {
    double *lp = L.rec + PCA_RW * i;
    for (int q = 0; q < 3; ++q) {
      lp[10 + q] = r.l[q];
      lp[22 + q] = fn[q];
      for (int k = 0; k < 3; ++k) lp[13 + 3 * q + k] = F[q][k];
    }
    L.stS[i] = (unsigned char)r.st;
  }
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    const double b[9] = {X[k][0].x, X[k][0].y, X[k][1].x, X[k][1].y, X[k][2].x,
                         X[k][2].y, X[k][3].x, X[k][3].y, X[k][4].x};
#pragma unroll
    for (int a = 0; a < 3; ++a) g[k][a] = fma(b[3 * a + 2], df[2], fma(b[3 * a + 1], df[1], fma(b[3 * a], df[0], g[k][a])));
  }
}

template <int K, int NS, int J>
__device__ inline void pca_slot(int nS, const double *__restrict__ Wb, PcaLds &L, int j_inner, int ln,
                                double (&g)[NS][3], double2 (&A)[NS][PGS_BLK / 2], double2 (&B)[NS][PGS_BLK / 2],
                                PcaRec &rA, PcaRec &rB, const icr_obstacle &obs, double t0, double t1, double h2) {
  const int last = nS - 1, end = min(nS, 64 * K + 64);
  for (int i = 64 * K; i < end; i += 2) {
    pca_rec(rB, L, min(i + 1, last));
    pca_step<K, NS, J>(i, A, rA, g, L, j_inner, ln, obs, t0, t1, h2);
    chain_load<NS>(A, Wb, min(i + 2, last), ln);
    if (i + 1 < end) {
      pca_rec(rA, L, min(i + 2, last));
      pca_step<K, NS, J>(i + 1, B, rB, g, L, j_inner, ln, obs, t0, t1, h2);
    }
    chain_load<NS>(B, Wb, min(i + 3, last), ln);
  }
}

template <int NS, int J>
__device__ __forceinline__ void pca_chain(int nS, const double *__restrict__ Wb, PcaLds &L, int j_inner,
                                          const icr_obstacle &obs, double t0, double t1, double h2) {
  const int ln = threadIdx.x & 63;
  double g[NS][3];
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    const int c = ln + 64 * k;
#pragma unroll
    for (int q = 0; q < 3; ++q) g[k][q] = c < nS ? L.P[3 * c + q] : 0.0;
  }
  const int last = nS - 1;
  double2 A[NS][PGS_BLK / 2], B[NS][PGS_BLK / 2];
  PcaRec rA, rB;
  chain_load<NS>(A, Wb, 0, ln);
  chain_load<NS>(B, Wb, min(1, last), ln);
  pca_rec(rA, L, 0);
  pca_slot<0, NS, J>(nS, Wb, L, j_inner, ln, g, A, B, rA, rB, obs, t0, t1, h2);
  if constexpr (NS > 1) pca_slot<1, NS, J>(nS, Wb, L, j_inner, ln, g, A, B, rA, rB, obs, t0, t1, h2);
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    const int c = ln + 64 * k;
    if (c < nS) {
#pragma unroll
      for (int q = 0; q < 3; ++q) L.P[3 * c + q] = g[k][q];
    }
  }
}

// A set of 65..128 contacts is swept by two waves as in chain_ring: wave w
// keeps the proximities of contacts 64 w .. 64 w + 63, solves those
// contacts while the other wave adds each published force change to its own
// proximities, then applies the other half's changes.  The applying wave
// takes the change as the published world force minus the force at the
// sweep's start, so every proximity receives the same products in the same
// order as in the one-wave sweep.
template <int J>
__device__ inline void pca_pair_solve(int b, int e, const double *__restrict__ Wb, PcaLds &L, int j_inner, int ln,
                                      int w, double (&g)[1][3], const icr_obstacle &obs, double t0, double t1,
                                      double h2) {
  if (b >= e) return;
  const int last = e - 1;
  double2 A[1][PGS_BLK / 2], B[1][PGS_BLK / 2];
  PcaRec rA, rB;
  ring_load<128>(A, Wb, b, 128, ln, w);
  ring_load<128>(B, Wb, min(b + 1, last), 128, ln, w);
  pca_rec(rA, L, b);
  for (int i = b; i < e; i += 2) {
    pca_rec(rB, L, min(i + 1, last));
    pca_step<0, 1, J>(i, A, rA, g, L, j_inner, ln, obs, t0, t1, h2);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    if (ln == 0) __hip_atomic_store(&L.cprog, i + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    ring_load<128>(A, Wb, min(i + 2, last), 128, ln, w);
    if (i + 1 < e) {
      pca_rec(rA, L, min(i + 2, last));
      pca_step<0, 1, J>(i + 1, B, rB, g, L, j_inner, ln, obs, t0, t1, h2);
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      if (ln == 0) __hip_atomic_store(&L.cprog, i + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    ring_load<128>(B, Wb, min(i + 3, last), 128, ln, w);
  }
}
__device__ inline void pca_pair_apply_one(int i, const double2 (&X)[1][PGS_BLK / 2], PcaLds &L, double (&g)[1][3]) {
  for (int spin = 0; __hip_atomic_load(&L.cprog, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) <= i; ++spin) {
    if (spin == RING_SPIN) {
      __hip_atomic_store(&L.perr, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      break;
    }
    if ((spin & 255) == 255 && __hip_atomic_load(&L.perr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != 0)
      break;
    __builtin_amdgcn_s_sleep(1);
  }
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  const double *rp = L.rec + PCA_RW * i + 22;
  const double d0 = rp[0] - L.f0[3 * i], d1 = rp[1] - L.f0[3 * i + 1], d2 = rp[2] - L.f0[3 * i + 2];
  const double bb[9] = {X[0][0].x, X[0][0].y, X[0][1].x, X[0][1].y, X[0][2].x,
                        X[0][2].y, X[0][3].x, X[0][3].y, X[0][4].x};
#pragma unroll
  for (int a = 0; a < 3; ++a) g[0][a] = fma(bb[3 * a + 2], d2, fma(bb[3 * a + 1], d1, fma(bb[3 * a], d0, g[0][a])));
}
__device__ inline void pca_pair_apply(int b, int e, const double *__restrict__ Wb, PcaLds &L, int ln, int w,
                                      double (&g)[1][3]) {
  if (b >= e) return;
  const int last = e - 1;
  double2 A[1][PGS_BLK / 2], B[1][PGS_BLK / 2];
  ring_load<128>(A, Wb, b, 128, ln, w);
  ring_load<128>(B, Wb, min(b + 1, last), 128, ln, w);
  for (int i = b; i < e; i += 2) {
    pca_pair_apply_one(i, A, L, g);
    ring_load<128>(A, Wb, min(i + 2, last), 128, ln, w);
    if (i + 1 < e) pca_pair_apply_one(i + 1, B, L, g);
    ring_load<128>(B, Wb, min(i + 3, last), 128, ln, w);
  }
}
template <int J>
__device__ __forceinline__ void pca_pair(int nS, const double *__restrict__ Wb, PcaLds &L, int j_inner,
                                         const icr_obstacle &obs, double t0, double t1, double h2, int w) {
  const int ln = threadIdx.x & 63, c = 64 * w + ln, h = min(64, nS);
  double g[1][3];
#pragma unroll
  for (int q = 0; q < 3; ++q) g[0][q] = c < nS ? L.P[3 * c + q] : 0.0;
  if (w == 0) {
    pca_pair_solve<J>(0, h, Wb, L, j_inner, ln, w, g, obs, t0, t1, h2);
    pca_pair_apply(h, nS, Wb, L, ln, w, g);
  } else {
    pca_pair_apply(0, h, Wb, L, ln, w, g);
    pca_pair_solve<J>(h, nS, Wb, L, j_inner, ln, w, g, obs, t0, t1, h2);
  }
  if (c < nS) {
#pragma unroll
    for (int q = 0; q < 3; ++q) L.P[3 * c + q] = g[0][q];
  }
}

// Exact proximity of a contact c outside S at its turn in the last sweep,
// by one wave (all lanes return it): Pset_c + h^2 sum_{b in S} W_H,cb
// (f_b^turn - f_b^set).
__device__ inline void pca_turn_proximity(int c, int nS, int m, const double *__restrict__ WH,
                                          const double *__restrict__ Pset, double h2, const PcaLds &L, int ln,
                                          double pt[3]) {
  double a[3] = {0.0, 0.0, 0.0};
  for (int q = ln; q < 3 * nS; q += 64) {
    const int b = L.Sidx[q / 3];
    const double fnew = L.rec[PCA_RW * (q / 3) + 22 + q % 3];
    const double d = ((b < c) ? fnew : L.f0[q]) - L.fset[q];
#pragma unroll
    for (int r = 0; r < 3; ++r) a[r] = fma(h2 * WH[(3L * c + r) * m + 3L * b + q % 3], d, a[r]);
  }
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    for (int o = 32; o > 0; o >>= 1) a[r] += __shfl_xor(a[r], o, 64);
    pt[r] = Pset[3 * c + r] + a[r];
  }
}

__global__ __launch_bounds__(PGS_NT) void k_pgs_pca(int nc, const StepCtx *__restrict__ ctx,
                                                    const double *__restrict__ WH, const double *__restrict__ pfree,
                                                    const double *__restrict__ pin, const double *__restrict__ pstart,
                                                    const double *__restrict__ mu, double h2, double *__restrict__ f,
                                                    double *__restrict__ C, double *__restrict__ lam,
                                                    int8_t *__restrict__ status, int max_sweeps, double tol,
                                                    int j_inner, int *__restrict__ sweeps_out,
                                                    double *__restrict__ eps_out, double *__restrict__ Wss,
                                                    double *__restrict__ Pset, double *__restrict__ gnSet,
                                                    double *__restrict__ swn, int *__restrict__ ctl) {
  extern __shared__ double lds_raw[];
  PcaLds &L = *reinterpret_cast<PcaLds *>(lds_raw);
  const int m = 3 * nc;
  const int tid = threadIdx.x, wv = tid >> 6, ln = tid & 63;
  const icr_obstacle obs = ctx->obs;
  const double t0 = ctx->t0, t1 = ctx->t0 + ctx->h;
  for (int c = tid; c < nc; c += PGS_NT) {
    const long d = 3L * c;
    swn[c] = sqrt(h2 * (WH[d * m + d] + WH[(d + 1) * m + d + 1] + WH[(d + 2) * m + d + 2]));
    L.inS[c] = 0;
  }
  for (int e = tid; e < m; e += PGS_NT) Pset[e] = pin[e];
  if (tid == 0) {
    ctl[0] = 0;
    ctl[1] = 0;
    L.stop = 0;
    L.perr = 0;
  }
  __syncthreads();
  int sweep = 0, nS = 0, nsp = 64;
  double eps = 0.0;
  bool need_build = true, first = true;
  while (sweep < max_sweeps) {
    if (need_build) {
      // proximity of the set's start state (given for the first set)
      if (!first) wg_sym_gemv_sparse<double>(nc, WH, pfree, f, f, h2, Pset, L.ulist, &L.nu, L.part);
      // normal gaps there; members: a force, a negative gap, or an earlier violation
      for (int c = tid; c < nc; c += PGS_NT) {
        const double pc[3] = {Pset[3 * c], Pset[3 * c + 1], Pset[3 * c + 2]};
        const double ps[3] = {pstart[3 * c], pstart[3 * c + 1], pstart[3 * c + 2]};
        double F[3][3], delta[3];
        contact_frame(obs, t0, t1, pc, ps, F, delta);
        gnSet[c] = delta[0];
        const bool nz = f[3 * c] != 0.0 || f[3 * c + 1] != 0.0 || f[3 * c + 2] != 0.0;
        if (nz || delta[0] < 0.0) L.inS[c] = 1;
      }
      __syncthreads();
      const int nwin = (nc + 63) / 64;
      for (int w = wv; w < nwin; w += PGS_NW) {
        const int c = 64 * w + ln;
        const unsigned long long bal = __ballot(c < nc && L.inS[c]);
        if (ln == 0) L.wcount[w] = __popcll(bal);
      }
      __syncthreads();
      if (tid == 0) {
        int acc = 0;
        for (int w = 0; w < nwin; ++w) {
          const int t = L.wcount[w];
          L.wcount[w] = acc;
          acc += t;
        }
        L.nS = acc;
      }
      __syncthreads();
      nS = L.nS;
      if (nS > PCA_MAX) {   // hand over: f and Pset hold the sweep-start state
        if (tid == 0) {
          ctl[0] = 1;
          ctl[1] = sweep;
        }
        return;
      }
      for (int w = wv; w < nwin; w += PGS_NW) {
        const int c = 64 * w + ln;
        const bool in = c < nc && L.inS[c];
        const unsigned long long bal = __ballot(in);
        if (in) L.Sidx[L.wcount[w] + __popcll(bal & ((1ull << ln) - 1ull))] = c;
      }
      __syncthreads();
      nsp = pgs_wave_pad(nS);
      for (int i = tid; i < nS; i += PGS_NT) {
        const long d = 3L * L.Sidx[i];
        double *rc = L.rec + PCA_RW * i;
        rc[0] = WH[d * m + d];
        rc[1] = WH[d * m + d + 1];
        rc[2] = WH[d * m + d + 2];
        rc[3] = WH[(d + 1) * m + d + 1];
        rc[4] = WH[(d + 1) * m + d + 2];
        rc[5] = WH[(d + 2) * m + d + 2];
        rc[6] = mu[L.Sidx[i]];
        for (int q = 0; q < 3; ++q) {
          rc[7 + q] = pstart[d + q];
          rc[22 + q] = f[d + q];
        }
      }
      for (int r = tid; r < 3 * nS; r += PGS_NT) {
        const long e = 3L * L.Sidx[r / 3] + r % 3;
        L.P[r] = Pset[e];
        L.fset[r] = f[e];
      }
      // h^2 W_H,SS blocked [i][c] (rows of contact c, columns of contact i),
      // diagonal blocks included
      const long nel = (long)nS * nsp * PGS_BLK;
      for (long e = tid; e < nel; e += PGS_NT) {
        const int j = (int)(e % PGS_BLK);
        const long ic = e / PGS_BLK;
        const int cc = (int)(ic % nsp), i = (int)(ic / nsp);
        double v = 0.0;
        if (j < 9 && cc < nS) v = h2 * WH[(3L * L.Sidx[cc] + j / 3) * m + 3L * L.Sidx[i] + j % 3];
        Wss[e] = v;
      }
      __threadfence_block();
      __syncthreads();
      need_build = false;
      first = false;
    }
    // ---- one sweep over S from its start state
    for (int r = tid; r < 3 * nS; r += PGS_NT) L.f0[r] = L.rec[PCA_RW * (r / 3) + 22 + r % 3];
    if (tid == 0) {
      L.flag = 0;
      L.nu = 0;
      L.cprog = 0;
    }
    __syncthreads();
    if (nS > 0) {
      if (nsp == 64) {
        if (wv == 0) {
          if (j_inner == 8)
            pca_chain<1, 8>(nS, Wss, L, j_inner, obs, t0, t1, h2);
          else
            pca_chain<1, 0>(nS, Wss, L, j_inner, obs, t0, t1, h2);
        }
      } else if (wv < 2) {
        if (j_inner == 8)
          pca_pair<8>(nS, Wss, L, j_inner, obs, t0, t1, h2, wv);
        else
          pca_pair<0>(nS, Wss, L, j_inner, obs, t0, t1, h2, wv);
      }
    }
    __syncthreads();
    // eps = |f_i - f_{i-1}| / |f_i| (forces outside S stay zero), and B
    double dpart = 0.0, bpart = 0.0, npart = 0.0;
    for (int i = tid; i < nS; i += PGS_NT) {
      const double *rc = L.rec + PCA_RW * i;
      double dnew = 0.0, dold = 0.0;
      for (int q = 0; q < 3; ++q) {
        const double fn = rc[22 + q], fo = L.f0[3 * i + q], fs = L.fset[3 * i + q];
        dpart += (fn - fo) * (fn - fo);
        npart += fn * fn;
        dnew += (fn - fs) * (fn - fs);
        dold += (fo - fs) * (fo - fs);
      }
      bpart += sqrt(h2 * (rc[0] + rc[3] + rc[5])) * sqrt(fmax(dnew, dold));
    }
    block_sum3(dpart, bpart, npart, L.red);
    if (tid == 0) {
      const double diff = sqrt(dpart), nf = sqrt(npart);
      eps = nf > 0.0 ? diff / nf : (diff == 0.0 ? 0.0 : INFINITY);
      if (L.perr) eps = NAN;   // the two-wave sweep lost its count: stop and report eps = NaN
      L.stop = (eps <= tol || L.perr) ? 1 : 0;
      L.red[0] = bpart * (1.0 + 1e-12);
    }
    __syncthreads();
    const double Bb = L.red[0];
    // ---- verify the skipped contacts
    for (int c = tid; c < nc; c += PGS_NT) {
      if (L.inS[c]) continue;
      const double g = gnSet[c], rb = swn[c] * Bb;
      if (!(g - rb > 1e-13 * (fabs(g) + rb))) L.ulist[atomicAdd(&L.nu, 1)] = c;
    }
    __syncthreads();
    const int nu = L.nu;
    for (int u = wv; u < nu; u += PGS_NW) {
      const int c = L.ulist[u];
      double pt[3];
      pca_turn_proximity(c, nS, m, WH, Pset, h2, L, ln, pt);
      if (ln == 0) {
        const double ps[3] = {pstart[3 * c], pstart[3 * c + 1], pstart[3 * c + 2]};
        double F[3][3], delta[3];
        contact_frame(obs, t0, t1, pt, ps, F, delta);
        if (delta[0] < 0.0) {
          L.inS[c] = 1;
          L.flag = 1;
        }
      }
    }
    __syncthreads();
    if (L.flag && !L.perr) {
      // a skipped contact was not a no-op: restart the sweep with a larger S
      for (int r = tid; r < 3 * nS; r += PGS_NT) f[3L * L.Sidx[r / 3] + r % 3] = L.f0[r];
      need_build = true;
      __threadfence_block();
      __syncthreads();
      continue;
    }
    ++sweep;
    if (L.stop) break;
  }
  // ---- results: S from its records; the others separate, with the frame at
  // their proximity at their turn in the last sweep
  for (int r = tid; r < 3 * nS; r += PGS_NT) {
    const long e = 3L * L.Sidx[r / 3] + r % 3;
    const double *rc = L.rec + PCA_RW * (r / 3);
    f[e] = rc[22 + r % 3];
    lam[e] = rc[10 + r % 3];
  }
  for (int i = tid; i < nS; i += PGS_NT) {
    const double *rc = L.rec + PCA_RW * i;
    for (int q = 0; q < 9; ++q) C[9L * L.Sidx[i] + q] = rc[13 + q];
    status[L.Sidx[i]] = (int8_t)L.stS[i];
  }
  for (int c = wv; c < nc; c += PGS_NW) {
    if (L.inS[c]) continue;
    double pt[3];
    pca_turn_proximity(c, nS, m, WH, Pset, h2, L, ln, pt);
    if (ln == 0) {
      const double ps[3] = {pstart[3 * c], pstart[3 * c + 1], pstart[3 * c + 2]};
      double F[3][3], delta[3];
      contact_frame(obs, t0, t1, pt, ps, F, delta);
      for (int r = 0; r < 3; ++r) {
        for (int q = 0; q < 3; ++q) C[9L * c + 3 * r + q] = F[r][q];
        lam[3 * c + r] = 0.0;
      }
      status[c] = (int8_t)ICR_SEPARATE;
    }
  }
  if (tid == 0) {
    *sweeps_out = sweep;
    *eps_out = eps;
  }
}

// ---- large active sets: block Gauss-Seidel over the whole GPU --------------
//
// When the active set outgrows the register chains (k_pgs_active hands over
// with ctl[0] = 1 and the sweep to resume in ctl[1]), the remaining sweeps
// run here, with the iterates of the sequential sweep: the contacts are
// taken in blocks of 128 in index order, and every block's force changes
// reach the gaps of all contacts, g += W~[:, block] dlambda (rows of the
// exactly symmetric W stand for its columns), before those contacts' turn.
// One cooperative launch with no grid barrier inside the sweeps:
//  - workgroup 0 (the lead) runs the chain of a block in wave 0 (the register
//    chain of the active-set kernel, which skips nothing: separated contacts
//    are solved and stay at zero); meanwhile waves 1-3 and 5-7 add the
//    block's force changes to the gaps of the NEXT block as the chain
//    publishes them, and wave 4 stages the next block's records and forces
//    in the other half of the LDS arrays.  So the next chain starts without
//    waiting for the rest of the GPU.
//  - the other workgroups push each published block's changes into all other
//    gap rows (64-row chunks, each chunk always owned by the same workgroup),
//    one block behind the lead, and report the last block they finished.
// The lead reads the next block's gaps only after every pushing workgroup
// finished the block before the current one, and reuses a block's change
// list (double-buffered) only after all of them read it.  Launched only when
// the stream is not being captured (else k_pgs_single continues).
constexpr int COOP_B = kPgsCoopB;   // contacts per block
constexpr int COOP_NT = PGS_NT;     // threads per workgroup
constexpr int COOP_MAXG = 128;      // workgroups of the launch at most
static_assert(3 * COOP_B == 6 * 64, "a block's gap rows are six 64-row chunks");
static_assert(COOP_NT == 512, "lead workgroup: chain wave, staging wave, six follower waves");
// sync words: [0] last published block, [1] stop, [2..3] changed contacts per
// list buffer, [4] a wait gave up, [8 + w] last block pushed by workgroup w
constexpr int COOP_SYNC_PUB = 0, COOP_SYNC_STOP = 1, COOP_SYNC_CNT = 2, COOP_SYNC_ERR = 4, COOP_SYNC_PROG = 8;
// Every wait is bounded (polls of device memory / of LDS, seconds in all,
// far beyond any legitimate wait): a wait that gives up sets the error word,
// every workgroup stops, and the call reports eps = NaN (not converged).
constexpr int COOP_SPIN_DEV = 1 << 22, COOP_SPIN_LDS = 1 << 24;
static_assert(COOP_SYNC_PROG + COOP_MAXG <= kPgsCoopSync, "sync words");
struct CoopArgs {
  int nc;
  const void *W;
  const double *d, *mu;
  double h2;
  double *lam;
  int8_t *status;
  int max_sweeps;
  double tol;
  int j_inner;
  int *sweeps_out;
  double *eps_out;
  const int *ctl;    // [0] handover, [1] first sweep
  double *g;         // [3 nc] gaps with the own term
  double *recAll;    // [nc * PGS_RW] records
  double *Wblk;      // [nblocks * COOP_B * COOP_B * PGS_BLK] blocked diagonal couplings
  double *dl;        // [2][3 COOP_B] force changes of the last two blocks
  int *chg;          // [2][COOP_B] their changed contacts (block-local)
  int *sync;         // [kPgsCoopSync] sync words
};

// Loads of data another workgroup of the launch wrote go to the
// device-coherent level, past this compute unit's own cache.
__device__ inline double ld_dev(const double *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline int ld_dev(const int *p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
__device__ inline void st_dev(int *p, int v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
__device__ inline int ld_wg(const int *p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP); }
__device__ inline void st_wg(int *p, int v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP); }

// y[r] = base[r] + h2 sum_k sum_a M[(3 c_k + a) m + r] v[3 k + a] for the rows
// of the 64-row chunks first, first + stride, ... outside [skip_lo, skip_hi):
// wave v takes list entries v, v + 8, ... (four at a time, twelve loads in
// flight); the eight partial sums are added in wave order.  W streams
// through with non-temporal loads, so that it does not evict the blocked
// couplings the chain reads.
template <class TW>
__device__ void coop_rows(int m, const TW *__restrict__ M, const int *list, int nlist, const double *vals,
                          int cbase, const double *base, double h2, double *y, double *part, int first, int stride,
                          int skip_lo, int skip_hi) {
  const int tid = threadIdx.x, wv = tid >> 6, ln = tid & 63;
  constexpr int NW = COOP_NT / 64;
  const int nchunk = (m + 63) / 64;
  for (int ch = first; ch < nchunk; ch += stride) {
    if (ch >= skip_lo && ch < skip_hi) continue;
    const int r = 64 * ch + ln;
    double a = 0.0;
    if (r < m) {
      for (int k = wv; k < nlist; k += 4 * NW) {
        double x[4][3];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int kk = k + NW * q;
          const long c3 = 3L * (cbase + list[kk < nlist ? kk : k]);
#pragma unroll
          for (int t = 0; t < 3; ++t) x[q][t] = kk < nlist ? (double)__builtin_nontemporal_load(M + (c3 + t) * m + r) : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int kk = k + NW * q;
          if (kk < nlist) {
            const double *vk = vals + 3 * kk;
            a = fma(x[q][0], vk[0], a);
            a = fma(x[q][1], vk[1], a);
            a = fma(x[q][2], vk[2], a);
          }
        }
      }
    }
    part[wv * 64 + ln] = a;
    __syncthreads();
    if (wv == 0 && r < m) {
      double t = 0.0;
      for (int w = 0; w < NW; ++w) t += part[w * 64 + ln];
      y[r] = ld_dev(base + r) + h2 * t;
    }
    __syncthreads();
  }
}

// Own-term-free gap of row e of the block staged at contact o of the LDS
// arrays: g - w lambda, w the contact's 3x3 block (record entries 0-5 =
// w00 w01 w02 w11 w12 w22), lambda its current force (entries 19-21).
__device__ inline double coop_own_free(const PgsLds &L, int o, int e, double g) {
  const double *rc = L.rec + PGS_RW * (o + e / 3);
  const int r = e % 3;
  const double w0 = r == 0 ? rc[0] : (r == 1 ? rc[1] : rc[2]);
  const double w1 = r == 0 ? rc[1] : (r == 1 ? rc[3] : rc[4]);
  const double w2 = r == 0 ? rc[2] : (r == 1 ? rc[4] : rc[5]);
  return g - (w0 * rc[19] + w1 * rc[20] + w2 * rc[21]);
}

// Lead workgroup (see above).
template <class TW>
__device__ void coop_lead(const CoopArgs &a, PgsLds &L, int sweep0) {
  const TW *__restrict__ W = static_cast<const TW *>(a.W);
  const int nc = a.nc, m = 3 * nc, nb = (nc + COOP_B - 1) / COOP_B;
  const double h2 = a.h2;
  const int tid = threadIdx.x, wv = tid >> 6, ln = tid & 63;
  const long blk_elems = (long)COOP_B * COOP_B * PGS_BLK;
  const int G = gridDim.x;
  const int total = (a.max_sweeps - sweep0) * nb;   // blocks to sweep
  int sweep = sweep0;
  double eps = 0.0;
  if (total > 0) {
    // block 0 staged at contact 0 of the LDS arrays
    {
      const int nB = min(COOP_B, nc);
      for (int e = tid; e < nB * 19; e += COOP_NT) L.rec[PGS_RW * (e / 19) + e % 19] = a.recAll[PGS_RW * (e / 19) + e % 19];
      for (int e = tid; e < 3 * nB; e += COOP_NT) {
        const double v = a.lam[e];
        L.rec[PGS_RW * (e / 3) + 19 + e % 3] = v;
        L.lamS0[e] = v;
      }
      __syncthreads();
      for (int e = tid; e < 3 * nB; e += COOP_NT) L.gS[e] = coop_own_free(L, 0, e, ld_dev(a.g + e));
      if (tid == 0) {
        L.cprog = 0;
        L.cflag = 0;
        L.stop = 0;
      }
      __syncthreads();
    }
    double dsum = 0.0, nl2 = 0.0;   // wave 0: sums of the sweep
    for (int s = 0; s < total; ++s) {
      const int b = s % nb, bn = (b + 1) % nb, p = s & 1;
      const int o = p ? COOP_B : 0, o1 = COOP_B - o;
      const int c0 = COOP_B * b, nB = min(COOP_B, nc - c0), nsp = pgs_wave_pad(nB);
      const int cn0 = COOP_B * bn, nBn = min(COOP_B, nc - cn0);
      if (wv == 0) {
        const double *Wb = a.Wblk + (long)b * blk_elems;
        if (a.j_inner == 8) {
          if (nsp == 64)
            chain_wave<1, 8, true>(nB, Wb, L, a.j_inner, o);
          else
            chain_wave<2, 8, true>(nB, Wb, L, a.j_inner, o);
        } else {
          if (nsp == 64)
            chain_wave<1, 0, true>(nB, Wb, L, a.j_inner, o);
          else
            chain_wave<2, 0, true>(nB, Wb, L, a.j_inner, o);
        }
      } else if (wv == 4) {
        // stage the next block's records and forces (unchanged by this chain)
        for (int e = ln; e < nBn * 19; e += 64)
          L.rec[PGS_RW * (o1 + e / 19) + e % 19] = a.recAll[PGS_RW * (long)(cn0 + e / 19) + e % 19];
        for (int e = ln; e < 3 * nBn; e += 64) {
          const double v = a.lam[3 * cn0 + e];
          L.rec[PGS_RW * (o1 + e / 3) + 19 + e % 3] = v;
          L.lamS0[3 * o1 + e] = v;
        }
        // every pushing workgroup finished block s - 1: the next block's gap
        // rows hold all earlier changes, and list buffer p ^ 1 is free
        for (int spin = 0;; ++spin) {
          bool ok = true;
          for (int w = 1 + ln; w < G; w += 64) ok &= ld_dev(a.sync + COOP_SYNC_PROG + w) >= s - 1;
          if (__ballot(!ok) == 0ull) break;
          if (spin == COOP_SPIN_DEV) {
            if (ln == 0) st_dev(a.sync + COOP_SYNC_ERR, 1);
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        if (ln == 0) st_wg(&L.cflag, 1);
      }
      // waves 1-3, 5-7: row f of the next block, f < 3 nBn
      const bool follower = wv != 0 && wv != 4;
      const int f = (wv < 4 ? wv - 1 : wv - 2) * 64 + ln;
      double acc = 0.0, gold = 0.0;
      bool have_g = false;
      if (follower) {
        const bool act = f < 3 * nBn;
        const long row = 3L * cn0 + (act ? f : 0);
        for (int i = 0; i < nB; i += 4) {
          double x[4][3];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const long c3 = 3L * (c0 + min(i + q, nB - 1));
#pragma unroll
            for (int t = 0; t < 3; ++t) x[q][t] = (double)__builtin_nontemporal_load(W + (c3 + t) * m + row);
          }
          const int need = min(i + 4, nB);
          for (int spin = 0; ld_wg(&L.cprog) < need; ++spin) {
            if (spin == COOP_SPIN_LDS) {
              st_dev(a.sync + COOP_SYNC_ERR, 1);
              break;
            }
            __builtin_amdgcn_s_sleep(1);
          }
          __atomic_signal_fence(__ATOMIC_SEQ_CST);
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            if (i + q < nB) {
              const double *rc = L.rec + PGS_RW * (o + i + q) + 19;
              const double *l0 = L.lamS0 + 3 * (o + i + q);
              acc = fma(x[q][0], rc[0] - l0[0], acc);
              acc = fma(x[q][1], rc[1] - l0[1], acc);
              acc = fma(x[q][2], rc[2] - l0[2], acc);
            }
          }
          if (!have_g && ld_wg(&L.cflag) != 0) {
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            gold = act ? ld_dev(a.g + row) : 0.0;
            have_g = true;
          }
        }
        if (!have_g) {
          for (int spin = 0; ld_wg(&L.cflag) == 0; ++spin) {
            if (spin == COOP_SPIN_LDS) {
              st_dev(a.sync + COOP_SYNC_ERR, 1);
              break;
            }
            __builtin_amdgcn_s_sleep(1);
          }
          __atomic_signal_fence(__ATOMIC_SEQ_CST);
          gold = act ? ld_dev(a.g + row) : 0.0;
        }
      }
      __syncthreads();
      if (wv == 0) {
        // new forces and statuses out, the changed contacts listed
        int cnt = 0;
        for (int i0 = 0; i0 < nB; i0 += 64) {
          const int i = i0 + ln;
          double d0 = 0.0, d1 = 0.0, d2 = 0.0, q2 = 0.0;
          if (i < nB) {
            const double *rc = L.rec + PGS_RW * (o + i);
            d0 = rc[19] - L.lamS0[3 * (o + i)];
            d1 = rc[20] - L.lamS0[3 * (o + i) + 1];
            d2 = rc[21] - L.lamS0[3 * (o + i) + 2];
            q2 = rc[19] * rc[19] + rc[20] * rc[20] + rc[21] * rc[21];
            a.lam[3 * (c0 + i)] = rc[19];
            a.lam[3 * (c0 + i) + 1] = rc[20];
            a.lam[3 * (c0 + i) + 2] = rc[21];
            a.status[c0 + i] = (int8_t)L.stS[o + i];
          }
          const bool ch = (d0 != 0.0) | (d1 != 0.0) | (d2 != 0.0);
          const unsigned long long bal = __ballot(ch);
          if (ch) {
            const int k = cnt + __popcll(bal & ((1ull << ln) - 1ull));
            a.chg[COOP_B * p + k] = i;
            a.dl[3 * COOP_B * p + 3 * k] = d0;
            a.dl[3 * COOP_B * p + 3 * k + 1] = d1;
            a.dl[3 * COOP_B * p + 3 * k + 2] = d2;
          }
          cnt += __popcll(bal);
          double sq = d0 * d0 + d1 * d1 + d2 * d2;
          for (int w = 32; w > 0; w >>= 1) {
            sq += __shfl_xor(sq, w, 64);
            q2 += __shfl_xor(q2, w, 64);
          }
          dsum += sq;   // same order every time
          nl2 += q2;
        }
        if (ln == 0) a.sync[COOP_SYNC_CNT + p] = cnt;
        int stop = 0;
        if (b == nb - 1) {
          // end of the sweep: eps = |lambda_i - lambda_{i-1}| / |lambda_i|
          const double diff = sqrt(dsum), nl = sqrt(nl2);
          eps = nl > 0.0 ? diff / nl : (diff == 0.0 ? 0.0 : INFINITY);
          ++sweep;
          stop = (eps <= a.tol || sweep >= a.max_sweeps) ? 1 : 0;
          dsum = nl2 = 0.0;
        }
        if (ld_dev(a.sync + COOP_SYNC_ERR) != 0) stop = 1;
        if (ln == 0) {
          L.stop = stop;
          if (stop) a.sync[COOP_SYNC_STOP] = 1;
        }
      } else if (follower && f < 3 * nBn) {
        const double gn = gold + h2 * acc;
        a.g[3L * cn0 + f] = gn;
        L.gS[3 * o1 + f] = coop_own_free(L, o1, f, gn);
      }
      __threadfence();
      if (tid == 0) {
        L.cprog = 0;
        L.cflag = 0;
      }
      __syncthreads();
      if (tid == 0) st_dev(a.sync + COOP_SYNC_PUB, s);
      if (L.stop) break;
    }
  } else if (tid == 0) {
    a.sync[COOP_SYNC_STOP] = 1;
    __threadfence();
    st_dev(a.sync + COOP_SYNC_PUB, 0);
  }
  if (tid == 0) {
    *a.sweeps_out = sweep;
    if (ld_dev(a.sync + COOP_SYNC_ERR) != 0)
      *a.eps_out = NAN;
    else if (total > 0)
      *a.eps_out = eps;
  }
}

// Pushing workgroups: block s's changes into every owned chunk of gap rows
// outside the next block, in block order, until the lead stops.
template <class TW>
__device__ void coop_push(const CoopArgs &a, PgsLds &L) {
  const TW *__restrict__ W = static_cast<const TW *>(a.W);
  const int nc = a.nc, m = 3 * nc, nb = (nc + COOP_B - 1) / COOP_B;
  const int tid = threadIdx.x;
  const int G = gridDim.x;
  for (int s = 0;; ++s) {
    if (tid == 0) {
      int stop = 0;
      for (int spin = 0; ld_dev(a.sync + COOP_SYNC_PUB) < s && (stop = ld_dev(a.sync + COOP_SYNC_STOP)) == 0; ++spin) {
        if (spin == COOP_SPIN_DEV) {
          st_dev(a.sync + COOP_SYNC_ERR, 1);
          stop = 1;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
      if (!stop) stop = ld_dev(a.sync + COOP_SYNC_STOP);
      L.stop = stop;
    }
    __syncthreads();
    if (L.stop) break;
    const int b = s % nb, bn = (b + 1) % nb, p = s & 1;
    const int nchg = ld_dev(a.sync + COOP_SYNC_CNT + p);
    for (int e = tid; e < nchg; e += COOP_NT) L.ulist[e] = ld_dev(a.chg + COOP_B * p + e);
    for (int e = tid; e < 3 * nchg; e += COOP_NT) L.lamSet[e] = ld_dev(a.dl + 3 * COOP_B * p + e);
    __syncthreads();
    if (nchg > 0)
      coop_rows<TW>(m, W, L.ulist, nchg, L.lamSet, COOP_B * b, a.g, a.h2, a.g, L.lamS, blockIdx.x - 1, G - 1, 6 * bn,
                    6 * bn + 6);
    __threadfence();
    __syncthreads();
    if (tid == 0) st_dev(a.sync + COOP_SYNC_PROG + blockIdx.x, s);
  }
}

template <class TW>
__global__ __launch_bounds__(COOP_NT) void k_pgs_coop(CoopArgs a) {
  extern __shared__ double lds_raw[];
  PgsLds &L = *reinterpret_cast<PgsLds *>(lds_raw);
  cooperative_groups::grid_group grid = cooperative_groups::this_grid();
  // control words written by the active-set kernel (an earlier launch)
  if (a.ctl[0] == 0) return;   // uniform: the active-set kernel finished the call
  const int sweep0 = a.ctl[1];
  const TW *__restrict__ W = static_cast<const TW *>(a.W);
  const int nc = a.nc, m = 3 * nc;
  const double h2 = a.h2;
  const int tid = threadIdx.x, wv = tid >> 6, ln = tid & 63;
  const int nb = (nc + COOP_B - 1) / COOP_B;
  const long blk_elems = (long)COOP_B * COOP_B * PGS_BLK;
  const long gthreads = (long)gridDim.x * COOP_NT, gt = (long)blockIdx.x * COOP_NT + tid;
  // ---- set-up, all workgroups: sync words, records, blocked couplings, gaps
  // at the resume state
  if (gt < kPgsCoopSync)
    a.sync[gt] = (gt == COOP_SYNC_STOP || gt == COOP_SYNC_CNT || gt == COOP_SYNC_CNT + 1 || gt == COOP_SYNC_ERR) ? 0 : -1;
  for (long c = gt; c < nc; c += gthreads) {
    double wb[3][3];
    for (int p = 0; p < 3; ++p)
      for (int q = 0; q < 3; ++q) wb[p][q] = h2 * (double)W[(3 * c + p) * m + 3 * c + q];
    double tmp[19];
    make_record(wb, a.mu[c], tmp);
    for (int q = 0; q < 19; ++q) a.recAll[PGS_RW * c + q] = tmp[q];
  }
  for (long e = gt; e < (long)nb * blk_elems; e += gthreads) {
    const int b = (int)(e / blk_elems);
    const long r = e % blk_elems;
    const int c0 = COOP_B * b, nB = min(COOP_B, nc - c0), nsp = pgs_wave_pad(nB);
    const int j = (int)(r % PGS_BLK);
    const long ic = r / PGS_BLK;
    const int c = (int)(ic % nsp), i = (int)(ic / nsp);
    double v = 0.0;
    if (i < nB && j < 9 && c < nB && c != i) v = h2 * (double)W[(3L * (c0 + c) + j / 3) * m + 3L * (c0 + i) + j % 3];
    if (i < nB) a.Wblk[(long)b * blk_elems + ((long)i * nsp + c) * PGS_BLK + j] = v;
  }
  {
    // contacts with a force, in every workgroup's LDS (order is fixed); the
    // running count is a wave-uniform register (the ballot is uniform)
    if (wv == 0) {
      int cnt = 0;
      for (int c0 = 0; c0 < nc; c0 += 64) {
        const int c = c0 + ln;
        const bool nz = c < nc && (a.lam[3 * c] != 0.0 || a.lam[3 * c + 1] != 0.0 || a.lam[3 * c + 2] != 0.0);
        const unsigned long long bal = __ballot(nz);
        if (nz) L.ulist[cnt + __popcll(bal & ((1ull << ln) - 1ull))] = c;
        cnt += __popcll(bal);
      }
      if (ln == 0) L.nu = cnt;
    }
    __syncthreads();
    const int nl = L.nu;
    // the force values in the order of the list, in LDS (reuses the set's gap area)
    double *vals = L.lamSet;
    double *part = L.lamS;
    for (int q0 = 0; q0 < nl; q0 += PGS_S3 / 3) {
      const int nq = min(PGS_S3 / 3, nl - q0);
      for (int e = tid; e < 3 * nq; e += COOP_NT) vals[e] = a.lam[3 * L.ulist[q0 + e / 3] + e % 3];
      __syncthreads();
      coop_rows<TW>(m, W, L.ulist + q0, nq, vals, 0, q0 == 0 ? a.d : a.g, h2, a.g, part, blockIdx.x, gridDim.x, 0, 0);
    }
    if (nl == 0)
      for (long r = gt; r < m; r += gthreads) a.g[r] = a.d[r];
  }
  __threadfence();
  grid.sync();
  if (blockIdx.x == 0)
    coop_lead<TW>(a, L, sweep0);
  else
    coop_push<TW>(a, L);
}

__global__ void k_world_force(int nc, const double *__restrict__ C, const double *__restrict__ lam,
                              double *__restrict__ f) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 3 * nc) return;
  f[e] = world_force(C, lam, e / 3, e % 3);
}

__global__ void k_zero(long n, double *__restrict__ x) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) x[i] = 0.0;
}

// Warm start of the next step (one workgroup): clear the forces of the
// previous step's contact nodes (count and ids on the device), store this
// step's world-frame forces on their nodes, keep their ids, advance the time.
// Pair contacts (the first npair contacts) keep their own forces.
__global__ __launch_bounds__(1024) void k_store_forces(int nc, const int *__restrict__ nodes,
                                                       const double *__restrict__ f, double *__restrict__ node_force,
                                                       int *__restrict__ prev_nodes, int *__restrict__ prev_nc,
                                                       StepCtx *__restrict__ ctx, int npair,
                                                       const double *__restrict__ fpair_new,
                                                       double *__restrict__ fpair) {
  for (int e = threadIdx.x; e < 3 * npair; e += blockDim.x) fpair[e] = fpair_new[e];
  const int pn = *prev_nc;
  for (int c = threadIdx.x; c < pn; c += blockDim.x) {
    const int v = prev_nodes[c];
    for (int a = 0; a < 3; ++a) node_force[3 * v + a] = 0.0;
  }
  __syncthreads();
  for (int c = threadIdx.x; c < nc; c += blockDim.x) {
    const int v = nodes[c];
    for (int a = 0; a < 3; ++a) node_force[3 * v + a] = f[3 * c + a];
  }
  __syncthreads();
  for (int c = threadIdx.x; c < nc; c += blockDim.x) prev_nodes[c] = nodes[c];
  if (threadIdx.x == 0) {
    *prev_nc = nc;
    ctx->t0 = ctx->t0 + ctx->h;
  }
}

// p = H q_k with q_k = q_free + h^2 A^-1 J^T lambda (Algorithm 2, steps 4-6).
__global__ void k_std_proximity(int nc, const int *__restrict__ nodes, const double *__restrict__ qf,
                                const double *__restrict__ sol, double h2, double *__restrict__ p) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  int v = nodes[c];
  for (int a = 0; a < 3; ++a) p[3 * c + a] = qf[3 * v + a] + h2 * sol[3 * v + a];
}

__global__ void k_set_ctx(StepCtx *ctx, icr_obstacle obs, int set_obs, double t0, int set_t, double h) {
  if (set_obs) ctx->obs = obs;
  if (set_t) ctx->t0 = t0;
  ctx->h = h;
}

__global__ void k_stamp(unsigned long long *ts, int slot) { ts[slot] = wall_clock64(); }


}  // namespace

void launch_select_contacts(icr_scene *s, int nc) {
  auto &C = s->con;
  const int P = s->pairs.count;   // pair contacts come first; the obstacle contacts follow them
  k_select<<<1, 1024, 0, s->stream>>>(C.count, C.d_cand, s->st.d_qfree, s->st.d_q, s->st.d_ctx, nc - P,
                                      C.d_mu_node, s->st.d_node_force, C.d_nodes_c + P, C.d_mu + P,
                                      C.d_pfree + 3L * P, C.d_pstart + 3L * P, C.d_f + 3L * P);
  ICR_LAUNCH_CHECK();
}

void launch_directions(icr_scene *s, int nc, bool first) {
  auto &C = s->con;
  const double *p = first ? C.d_pfree : C.d_p;
  k_directions<<<cdiv(nc, 128), 128, 0, s->stream>>>(nc, s->st.d_ctx, p, C.d_pfree, C.d_pstart, C.d_f, C.d_C,
                                                     C.d_dk, C.d_lam, s->pairs.count, s->pairs.d_normal);
  ICR_LAUNCH_CHECK();
}

// Pair contacts 0..P-1 of a step: p_free = H q_free, p_start = H q over their
// slots, friction, warm start from the pair's previous force, node id -1;
// and the node list of the W_H build: the pairs' distinct nodes, then the
// step's obstacle contact nodes (contacts P..nc-1).
__global__ void k_pair_points(int P, int nc, int nup, const int *__restrict__ slot_node,
                              const double *__restrict__ w, const double *__restrict__ qf,
                              const double *__restrict__ q, const double *__restrict__ mu_pair,
                              const double *__restrict__ fpair, const int *__restrict__ pair_nodes,
                              int *__restrict__ nodes_c, double *__restrict__ mu_c, double *__restrict__ pfree,
                              double *__restrict__ pstart, double *__restrict__ finit, int *__restrict__ unodes) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < P) {
    double a[3] = {0, 0, 0}, b[3] = {0, 0, 0};
    for (int k = 0; k < 4; ++k) {
      const int v = slot_node[4 * t + k];
      if (v < 0) continue;
      const double wk = w[4 * t + k];
      for (int x = 0; x < 3; ++x) {
        a[x] = fma(wk, qf[3 * v + x], a[x]);
        b[x] = fma(wk, q[3 * v + x], b[x]);
      }
    }
    for (int x = 0; x < 3; ++x) {
      pfree[3 * t + x] = a[x];
      pstart[3 * t + x] = b[x];
      finit[3 * t + x] = fpair[3 * t + x];
    }
    mu_c[t] = mu_pair[t];
    nodes_c[t] = -1;
  }
  if (t < nup) unodes[t] = pair_nodes[t];
  if (t >= nup && t < nup + nc - P) unodes[t] = nodes_c[P + t - nup];
}

// Force on every node of the W_H build (H_w^T f): a pair node sums weight x
// force over the pair slots that name it (CSR in slot order), an obstacle
// contact's node takes that contact's force.
__global__ void k_node_forces(int nup, int nu, int P, const int *__restrict__ csr_ptr,
                              const int *__restrict__ csr_slot, const double *__restrict__ w,
                              const double *__restrict__ f, double *__restrict__ fu) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= nu) return;
  double a[3] = {0, 0, 0};
  if (u < nup) {
    for (int e = csr_ptr[u]; e < csr_ptr[u + 1]; ++e) {
      const int sl = csr_slot[e], c = sl / 4;
      for (int x = 0; x < 3; ++x) a[x] = fma(w[sl], f[3 * c + x], a[x]);
    }
  } else {
    const int c = P + u - nup;
    for (int x = 0; x < 3; ++x) a[x] = f[3 * c + x];
  }
  for (int x = 0; x < 3; ++x) fu[3 * u + x] = a[x];
}

void launch_pair_points(icr_scene *s, int nc) {
  auto &C = s->con;
  auto &Pr = s->pairs;
  const int n = std::max(Pr.count, Pr.nu + nc - Pr.count);
  k_pair_points<<<cdiv(n, 256), 256, 0, s->stream>>>(Pr.count, nc, Pr.nu, Pr.d_slot_node, Pr.d_w, s->st.d_qfree,
                                                     s->st.d_q, Pr.d_mu, Pr.d_force, Pr.d_nodes, C.d_nodes_c,
                                                     C.d_mu, C.d_pfree, C.d_pstart, C.d_f, Pr.d_unodes);
  ICR_LAUNCH_CHECK();
}

void launch_node_forces(icr_scene *s, int nc, const double *f, double *fu) {
  auto &Pr = s->pairs;
  const int nu = Pr.nu + nc - Pr.count;
  k_node_forces<<<cdiv(nu, 256), 256, 0, s->stream>>>(Pr.nu, nu, Pr.count, Pr.d_csr_ptr, Pr.d_csr_slot, Pr.d_w,
                                                      f, fu);
  ICR_LAUNCH_CHECK();
}

template <class TW>
void launch_update_W(hipStream_t st, int nc, const TW *WH, const double *Cm, TW *W) {
  long nb = (long)nc * nc;
  k_update_W<TW><<<(unsigned)((nb + 255) / 256), 256, 0, st>>>(nc, WH, Cm, W);
  ICR_LAUNCH_CHECK();
}
template void launch_update_W<double>(hipStream_t, int, const double *, const double *, double *);
template void launch_update_W<float>(hipStream_t, int, const float *, const double *, float *);

template <class TW>
void launch_pgs(hipStream_t st, int nc, const TW *W, const double *d, const double *mu, double h, double *lam,
                int8_t *status, int max_sweeps, double tol, int j_inner, int *sweeps_dev, double *eps_dev,
                const PgsWork &wk) {
  const int m = 3 * nc;
  // g0 = d + W~ lambda over the contacts with a warm-start force
  k_sym_gemv_sparse<TW><<<cdiv(m, 64), SG_NT, 0, st>>>(nc, W, d, lam, h * h, wk.g, nullptr, nullptr, nullptr);
  ICR_LAUNCH_CHECK();
  k_pgs_gather<TW><<<512, 256, 0, st>>>(nc, W, wk.g, lam, mu, h * h, wk.Sidx, wk.nS, wk.gnSet, wk.swn, wk.Wss, wk.rec,
                                    wk.gS);
  ICR_LAUNCH_CHECK();
  k_pgs_active<TW><<<1, PGS_NT, sizeof(PgsLds), st>>>(nc, W, d, wk.g, mu, h * h, lam, status, max_sweeps, tol, j_inner,
                                                sweeps_dev, eps_dev, wk.Wss, wk.gnSet, wk.swn, wk.ctl, wk.Sidx,
                                                wk.nS, wk.rec, wk.gS);
  ICR_LAUNCH_CHECK();
  // continues only if the active set outgrew the compact path: block
  // Gauss-Seidel over the whole GPU, or (under stream capture, or without
  // its buffers) the single-workgroup sweep
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  ICR_HIP(hipStreamIsCapturing(st, &cap));
  const int G = coop_grid();
  if (nc > PGS_WAVE_MAX && wk.Wblk != nullptr && G > 1 && cap == hipStreamCaptureStatusNone) {
    CoopArgs a{nc, W, d, mu, h * h, lam, status, max_sweeps, tol, j_inner, sweeps_dev, eps_dev, wk.ctl, wk.g,
               wk.recAll, wk.Wblk, wk.dl, wk.chg, wk.csync};
    void *args[] = {&a};
    ICR_HIP(hipLaunchCooperativeKernel((const void *)k_pgs_coop<TW>, dim3(G), dim3(COOP_NT), args, sizeof(PgsLds), st));
  } else {
    k_pgs_single<TW><<<1, 1024, pgs_single_lds(nc), st>>>(nc, W, d, nullptr, mu, h * h, lam, status, max_sweeps, tol,
                                                          j_inner, sweeps_dev, eps_dev, wk.ctl);
    ICR_LAUNCH_CHECK();
  }
}
template void launch_pgs<double>(hipStream_t, int, const double *, const double *, const double *, double, double *,
                                 int8_t *, int, double, int, int *, double *, const PgsWork &);
template void launch_pgs<float>(hipStream_t, int, const float *, const double *, const double *, double, double *,
                                int8_t *, int, double, int, int *, double *, const PgsWork &);

void launch_pgs_per_constraint(hipStream_t st, int nc, const StepCtx *ctx, const double *WH, const double *pfree,
                               const double *p, const double *pstart, const double *mu, double h, double *f,
                               double *Cm, double *lam, int8_t *status, int max_sweeps, double tol, int j_inner,
                               int *sweeps_dev, double *eps_dev, const PgsWork &wk) {
  // the register chain over the contacts that can change, then (only if
  // their set outgrew the chain) the one-workgroup sweep from that state
  k_pgs_pca<<<1, PGS_NT, sizeof(PcaLds), st>>>(nc, ctx, WH, pfree, p, pstart, mu, h * h, f, Cm, lam, status,
                                               max_sweeps, tol, j_inner, sweeps_dev, eps_dev, wk.Wss, wk.g, wk.gnSet,
                                               wk.swn, wk.ctl);
  ICR_LAUNCH_CHECK();
  k_pgs_pc<<<1, 1024, pgs_pc_lds(nc), st>>>(nc, ctx, WH, wk.g, pstart, mu, h * h, f, Cm, lam, status, max_sweeps, tol,
                                           j_inner, sweeps_dev, eps_dev, wk.ctl);
  ICR_LAUNCH_CHECK();
}

namespace {
int g_coop_grid[64];   // per device: workgroups of the cooperative PGS launch (0 = not available)
}

int coop_grid() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  return g_coop_grid[dev];
}

void pgs_prepare() {
  // kernel attributes are set once per device
  static std::mutex mtx;
  static unsigned long long done = 0;
  int dev = 0;
  ICR_HIP(hipGetDevice(&dev));
  const unsigned long long bit = 1ull << (dev & 63);
  std::lock_guard<std::mutex> lock(mtx);
  if (done & bit) return;
  ICR_HIP(hipFuncSetAttribute((const void *)k_pgs_active<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)sizeof(PgsLds)));
  ICR_HIP(hipFuncSetAttribute((const void *)k_pgs_active<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)sizeof(PgsLds)));
  ICR_HIP(hipFuncSetAttribute((const void *)k_pgs_single<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)pgs_single_lds(PGS_MAX_NC)));
  ICR_HIP(hipFuncSetAttribute((const void *)k_pgs_single<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)pgs_single_lds(PGS_MAX_NC)));
  ICR_HIP(hipFuncSetAttribute((const void *)k_pgs_pc, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)pgs_pc_lds(PGS_MAX_NC)));
  ICR_HIP(hipFuncSetAttribute((const void *)k_pgs_coop<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)sizeof(PgsLds)));
  ICR_HIP(hipFuncSetAttribute((const void *)k_newton_batch, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)sizeof(PgsLds)));
  ICR_HIP(hipFuncSetAttribute((const void *)k_pgs_pca, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)sizeof(PcaLds)));
  ICR_HIP(hipFuncSetAttribute((const void *)k_pgs_coop<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)sizeof(PgsLds)));
  // cooperative launch: at most one workgroup per compute unit (its LDS),
  // 128 workgroups at most (enough to stream the gap updates)
  int coop = 0, cus = 0, per_cu = 0;
  g_coop_grid[dev & 63] = 0;
  if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) == hipSuccess && coop &&
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_pgs_coop<double>, COOP_NT,
                                                   sizeof(PgsLds)) == hipSuccess &&
      per_cu > 0)
    g_coop_grid[dev & 63] = std::min(128, per_cu * cus);
  done |= bit;
}

void launch_newton_batch(hipStream_t st, const NewtonTask *tasks, const NewtonBatchIdx &ids) {
  if (ids.n < 1 || ids.n > kNewtonBatchMax) throw std::runtime_error("batched Newton loop: 1..64 scenes");
  pgs_prepare();
  k_newton_batch<<<ids.n, PGS_NT, sizeof(PgsLds), st>>>(tasks, ids);
  ICR_LAUNCH_CHECK();
}

void launch_world_force(hipStream_t st, int nc, const double *Cm, const double *lam, double *f) {
  k_world_force<<<cdiv(3 * nc, 256), 256, 0, st>>>(nc, Cm, lam, f);
  ICR_LAUNCH_CHECK();
}

template <class TW>
void launch_world_force_proximity(hipStream_t st, int nc, const double *Cm, const double *lam, double *f,
                                  const TW *WH, const double *p_free, double h, double *p) {
  const int m = 3 * nc;
  // f = C^T lambda and p = p_free + h^2 W_H f in one launch
  k_sym_gemv_sparse<TW><<<cdiv(m, 64), SG_NT, 0, st>>>(nc, WH, p_free, nullptr, h * h, p, Cm, lam, f);
  ICR_LAUNCH_CHECK();
}
template void launch_world_force_proximity<double>(hipStream_t, int, const double *, const double *, double *,
                                                   const double *, const double *, double, double *);
template void launch_world_force_proximity<float>(hipStream_t, int, const double *, const double *, double *,
                                                  const float *, const double *, double, double *);

template <class TW>
void launch_proximity(hipStream_t st, int nc, const TW *WH, const double *p_free, const double *f, double h,
                      double *p) {
  const int m = 3 * nc;
  // p = p_free + h^2 W_H f; f is zero at separated contacts
  k_sym_gemv_sparse<TW><<<cdiv(m, 64), SG_NT, 0, st>>>(nc, WH, p_free, f, h * h, p, nullptr, nullptr, nullptr);
  ICR_LAUNCH_CHECK();
}
template void launch_proximity<double>(hipStream_t, int, const double *, const double *, const double *, double,
                                       double *);
template void launch_proximity<float>(hipStream_t, int, const float *, const double *, const double *, double,
                                      double *);

void launch_set_ctx(icr_scene *s, const icr_obstacle *obs, const double *t0) {
  icr_obstacle o{};
  if (obs) o = *obs;
  k_set_ctx<<<1, 1, 0, s->stream>>>(s->st.d_ctx, o, obs ? 1 : 0, t0 ? *t0 : 0.0, t0 ? 1 : 0, s->mesh.h);
  ICR_LAUNCH_CHECK();
}

void launch_stamp(icr_scene *s, int slot) {
  k_stamp<<<1, 1, 0, s->stream>>>(s->st.d_stamps, slot);
  ICR_LAUNCH_CHECK();
}

void launch_standard_proximity(icr_scene *s, int nc) {
  const double h = s->mesh.h;
  k_std_proximity<<<cdiv(nc, 128), 128, 0, s->stream>>>(nc, s->con.d_nodes_c, s->st.d_qfree, s->st.d_sol, h * h,
                                                         s->con.d_p);
  ICR_LAUNCH_CHECK();
}

void launch_store_forces(icr_scene *s, int nc) {
  auto &S = s->st;
  const int P = s->pairs.count;
  k_store_forces<<<1, 1024, 0, s->stream>>>(nc - P, s->con.d_nodes_c + P, s->con.d_f + 3L * P, S.d_node_force,
                                            S.d_prev_nodes, S.d_prev_nc, S.d_ctx, P, s->con.d_f,
                                            s->pairs.d_force);
  ICR_LAUNCH_CHECK();
}

}  // namespace icr
