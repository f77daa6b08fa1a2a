// Linear-tetrahedron FE assembly and the free-motion right-hand side
// (Sec. "Implicit time integration", Eq. 4-5) on the device.
//
// Element matrices are formed one thread per tetrahedron; the 3x3 blocks of
// K and A are then summed one thread per block from a host-built list of
// element contributions in ascending element order (deterministic, no atomics).
#include "scene.hpp"

namespace icr {

namespace {

// K_e[ai, bj] = V (lam g_a,i g_b,j + mu g_a,j g_b,i + mu delta_ij g_a.g_b),
// g_a the gradient of the linear shape function of vertex a.
__global__ void k_element(int T, const double *__restrict__ nodes, const int *__restrict__ tets,
                          const double *__restrict__ E, const double *__restrict__ nu, double *__restrict__ Ke,
                          double *__restrict__ vol, int *__restrict__ err) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T) return;
  double x[4][3];
  for (int a = 0; a < 4; ++a) {
    int v = tets[4 * t + a];
    for (int i = 0; i < 3; ++i) x[a][i] = nodes[3 * v + i];
  }
  // Dm columns e_c = x_{c+1} - x_0 ; Dm[r][c]
  double D[3][3];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) D[r][c] = x[c + 1][r] - x[0][r];
  double c00 = D[1][1] * D[2][2] - D[1][2] * D[2][1];
  double c01 = D[1][2] * D[2][0] - D[1][0] * D[2][2];
  double c02 = D[1][0] * D[2][1] - D[1][1] * D[2][0];
  double det = D[0][0] * c00 + D[0][1] * c01 + D[0][2] * c02;
  double V = det / 6.0;
  vol[t] = V;
  if (!(V > 0.0)) atomicMin(err, t);
  // inverse of Dm: rows are gradients of barycentric coordinates 1..3
  double inv[3][3];
  inv[0][0] = c00 / det;
  inv[1][0] = c01 / det;
  inv[2][0] = c02 / det;
  inv[0][1] = (D[0][2] * D[2][1] - D[0][1] * D[2][2]) / det;
  inv[1][1] = (D[0][0] * D[2][2] - D[0][2] * D[2][0]) / det;
  inv[2][1] = (D[0][1] * D[2][0] - D[0][0] * D[2][1]) / det;
  inv[0][2] = (D[0][1] * D[1][2] - D[0][2] * D[1][1]) / det;
  inv[1][2] = (D[0][2] * D[1][0] - D[0][0] * D[1][2]) / det;
  inv[2][2] = (D[0][0] * D[1][1] - D[0][1] * D[1][0]) / det;
  double g[4][3];
  for (int i = 0; i < 3; ++i) {
    g[1][i] = inv[0][i];
    g[2][i] = inv[1][i];
    g[3][i] = inv[2][i];
    g[0][i] = -(inv[0][i] + inv[1][i] + inv[2][i]);
  }
  double e = E[t], p = nu[t];
  double lam = e * p / ((1.0 + p) * (1.0 - 2.0 * p));
  double mu = e / (2.0 * (1.0 + p));
  double *K = Ke + (long)t * 144;
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) {
      double gg = g[a][0] * g[b][0] + g[a][1] * g[b][1] + g[a][2] * g[b][2];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          double v = lam * g[a][i] * g[b][j] + mu * g[a][j] * g[b][i];
          if (i == j) v += mu * gg;
          K[(3 * a + i) * 12 + 3 * b + j] = V * v;
        }
    }
}

// Lumped mass: m_i = sum over incident elements of rho V / 4, element order.
__global__ void k_mass(int N, const int *__restrict__ nt_ptr, const int *__restrict__ nt,
                       const double *__restrict__ vol, double rho, double *__restrict__ mass) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double m = 0.0;
  for (int e = nt_ptr[i]; e < nt_ptr[i + 1]; ++e) m += rho * vol[nt[e]] / 4.0;
  mass[i] = m;
}

// K and A = M + h (alpha M + beta K) + h^2 K per 3x3 block; clamped nodes get
// identity diagonal blocks and zero coupling blocks.
__global__ void k_blocks(int nnzb, const int *__restrict__ bsr_row, const int *__restrict__ bsr_col,
                         const int *__restrict__ contrib_ptr, const int *__restrict__ contrib,
                         const double *__restrict__ Ke, const double *__restrict__ mass,
                         const uint8_t *__restrict__ fixed, double h, double alpha, double beta,
                         double *__restrict__ Kb, double *__restrict__ Ab) {
  int blk = blockIdx.x * blockDim.x + threadIdx.x;
  if (blk >= nnzb) return;
  double k[9];
  for (int q = 0; q < 9; ++q) k[q] = 0.0;
  for (int e = contrib_ptr[blk]; e < contrib_ptr[blk + 1]; ++e) {
    int c = contrib[e];
    int t = c >> 4, a = (c >> 2) & 3, b = c & 3;
    const double *K = Ke + (long)t * 144;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) k[3 * i + j] += K[(3 * a + i) * 12 + 3 * b + j];
  }
  int r = bsr_row[blk], c = bsr_col[blk];
  for (int q = 0; q < 9; ++q) Kb[9 * blk + q] = k[q];
  bool clamp = fixed[r] || fixed[c];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double m = (r == c && i == j) ? mass[r] : 0.0;
      double a = m + h * (alpha * m + beta * k[3 * i + j]) + (h * h) * k[3 * i + j];
      if (clamp) a = (r == c && i == j) ? 1.0 : 0.0;
      Ab[9 * blk + 3 * i + j] = a;
    }
}

// b = h M g - h (K (q - q_rest) + alpha M v + beta K v) - h^2 K v, zero at clamped DOFs.
__global__ void k_free_rhs(int N, const int *__restrict__ bsr_ptr, const int *__restrict__ bsr_col,
                           const double *__restrict__ Kb, const double *__restrict__ mass,
                           const uint8_t *__restrict__ fixed, const double *__restrict__ q,
                           const double *__restrict__ qrest, const double *__restrict__ v, double h, double alpha,
                           double beta, double gx, double gy, double gz, double *__restrict__ b) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double ku[3] = {0, 0, 0}, kv[3] = {0, 0, 0};
  for (int e = bsr_ptr[i]; e < bsr_ptr[i + 1]; ++e) {
    int c = bsr_col[e];
    const double *K = Kb + 9 * (long)e;
    double u0 = q[3 * c] - qrest[3 * c], u1 = q[3 * c + 1] - qrest[3 * c + 1], u2 = q[3 * c + 2] - qrest[3 * c + 2];
    double v0 = v[3 * c], v1 = v[3 * c + 1], v2 = v[3 * c + 2];
    for (int a = 0; a < 3; ++a) {
      ku[a] += K[3 * a] * u0 + K[3 * a + 1] * u1 + K[3 * a + 2] * u2;
      kv[a] += K[3 * a] * v0 + K[3 * a + 1] * v1 + K[3 * a + 2] * v2;
    }
  }
  double g[3] = {gx, gy, gz};
  double m = mass[i];
  for (int a = 0; a < 3; ++a) {
    double vi = v[3 * i + a];
    double f = ku[a] + (alpha * m * vi + beta * kv[a]);
    double val = h * (m * g[a]) - h * f - (h * h) * kv[a];
    b[3 * i + a] = fixed[i] ? 0.0 : val;
  }
}

__global__ void k_qfree(int n, const double *__restrict__ q, const double *__restrict__ v,
                        const double *__restrict__ dv, double h, double *__restrict__ qf) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) qf[i] = q[i] + h * (v[i] + dv[i]);
}

// dv = dv_free + h * sol; v += dv; q += h v  (Eq. 20, Algorithm 1 last loop)
__global__ void k_integrate(int n, double *__restrict__ q, double *__restrict__ v, const double *__restrict__ dvf,
                            const double *__restrict__ sol, double h) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double dv = dvf[i] + h * sol[i];
  double vn = v[i] + dv;
  v[i] = vn;
  q[i] = q[i] + h * vn;
}

}  // namespace

void launch_element_matrices(icr_scene *s) {
  auto &m = s->mesh;
  k_element<<<cdiv(m.T, 128), 128, 0, s->stream>>>(m.T, m.d_nodes, m.d_tets, m.d_E, m.d_nu, m.d_Ke, m.d_vol,
                                                   m.d_err);
  ICR_LAUNCH_CHECK();
  k_mass<<<cdiv(m.N, 256), 256, 0, s->stream>>>(m.N, m.d_nt_ptr, m.d_nt, m.d_vol, m.rho, m.d_mass);
  ICR_LAUNCH_CHECK();
}

void launch_assemble_blocks(icr_scene *s) {
  auto &m = s->mesh;
  k_blocks<<<cdiv(m.nnzb, 128), 128, 0, s->stream>>>(m.nnzb, m.d_bsr_row, m.d_bsr_col, m.d_contrib_ptr,
                                                     m.d_contrib, m.d_Ke, m.d_mass, m.d_fixed, m.h, m.alpha,
                                                     m.beta, m.d_K, m.d_A);
  ICR_LAUNCH_CHECK();
}

void launch_free_rhs(icr_scene *s, const double *q, const double *v, double *b) {
  auto &m = s->mesh;
  k_free_rhs<<<cdiv(m.N, 128), 128, 0, s->stream>>>(m.N, m.d_bsr_ptr, m.d_bsr_col, m.d_K, m.d_mass, m.d_fixed,
                                                     q, s->st.d_qrest, v, m.h, m.alpha, m.beta, m.grav[0],
                                                     m.grav[1], m.grav[2], b);
  ICR_LAUNCH_CHECK();
}

void launch_axpy_qfree(icr_scene *s) {
  int n = s->mesh.n;
  k_qfree<<<cdiv(n, 256), 256, 0, s->stream>>>(n, s->st.d_q, s->st.d_v, s->st.d_dvfree, s->mesh.h,
                                                 s->st.d_qfree);
  ICR_LAUNCH_CHECK();
}

void launch_integrate(icr_scene *s) {
  int n = s->mesh.n;
  k_integrate<<<cdiv(n, 256), 256, 0, s->stream>>>(n, s->st.d_q, s->st.d_v, s->st.d_dvfree, s->st.d_sol,
                                                     s->mesh.h);
  ICR_LAUNCH_CHECK();
}

}  // namespace icr
