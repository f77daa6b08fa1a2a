// C ABI entry points (include/icr.h): argument checks, host planning, and the
// launch sequence of each call on the scene's stream.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <exception>
#include <numeric>

#include "scene.hpp"
#include "server_hooks.hpp"

using namespace icr;

namespace {

struct ArgError : std::runtime_error {
  using std::runtime_error::runtime_error;
};
struct StateError : std::runtime_error {
  using std::runtime_error::runtime_error;
};
struct SpdError : std::runtime_error {
  using std::runtime_error::runtime_error;
};

template <class F>
icr_status guarded(icr_scene *s, F &&body) {
  if (!s) return ICR_E_ARG;
  s->err.clear();
  try {
    return body();
  } catch (const ArgError &e) {
    s->err = e.what();
    return ICR_E_ARG;
  } catch (const StateError &e) {
    s->err = e.what();
    return ICR_E_STATE;
  } catch (const SpdError &e) {
    s->err = e.what();
    return ICR_E_NOT_SPD;
  } catch (const HipError &e) {
    s->err = e.what();
    return (e.code == hipErrorOutOfMemory) ? ICR_E_OOM : ICR_E_HIP;
  } catch (const std::bad_alloc &) {
    s->err = "host allocation failed";
    return ICR_E_OOM;
  } catch (const std::exception &e) {
    s->err = e.what();
    return ICR_E_HIP;
  }
}

#define REQUIRE(cond, msg) \
  do {                     \
    if (!(cond)) throw ArgError(msg); \
  } while (0)

void ensure_contact_buffers(icr_scene *s, int nc) {
  auto &C = s->con;
  if (nc <= C.nc_cap) return;
  s->epoch++;
  ICR_HIP(hipStreamSynchronize(s->stream));
  C.arena.release();
  const long m = 3L * nc;
  C.d_nodes_c = C.arena.alloc<int>(nc);
  C.d_mu = C.arena.alloc<double>(nc);
  C.d_pfree = C.arena.alloc<double>(m);
  C.d_pstart = C.arena.alloc<double>(m);
  C.d_p = C.arena.alloc<double>(m);
  C.d_C = C.arena.alloc<double>(9L * nc);
  C.d_dk = C.arena.alloc<double>(m);
  C.d_lam = C.arena.alloc<double>(m);
  C.d_f = C.arena.alloc<double>(m);
  C.d_WH = C.arena.alloc<double>(m * m);
  C.d_W = C.arena.alloc<double>(m * m);
  C.d_WH32 = C.arena.alloc<float>(m * m);
  C.d_W32 = C.arena.alloc<float>(m * m);
  C.pgs.g = C.arena.alloc<double>(m);
  C.pgs.Wss = C.arena.alloc<double>(pgs_wss_elems(nc));
  C.pgs.gnSet = C.arena.alloc<double>(nc);
  C.pgs.swn = C.arena.alloc<double>(nc);
  C.pgs.Sidx = C.arena.alloc<int>(nc);
  C.pgs.nS = C.arena.alloc<int>(1);
  C.pgs.rec = C.arena.alloc<double>(pgs_rec_elems(nc));
  C.pgs.gS = C.arena.alloc<double>(pgs_rec_elems(nc));
  C.pgs.ctl = C.arena.alloc<int>(4);
  if (nc > kPgsWaveMax) {
    C.pgs.recAll = C.arena.alloc<double>((size_t)nc * kPgsRecWidth);
    C.pgs.Wblk = C.arena.alloc<double>(pgs_coop_blk_elems(nc));
    C.pgs.dl = C.arena.alloc<double>(2 * 3 * kPgsCoopB);
    C.pgs.chg = C.arena.alloc<int>(2 * kPgsCoopB);
    C.pgs.csync = C.arena.alloc<int>(kPgsCoopSync);
  } else {
    C.pgs.recAll = C.pgs.Wblk = C.pgs.dl = nullptr;
    C.pgs.chg = C.pgs.csync = nullptr;
  }
  pgs_prepare();
  C.d_status = C.arena.alloc<int8_t>(nc);
  C.d_sweeps = C.arena.alloc<int>(kMaxNewton);
  C.d_eps = C.arena.alloc<double>(kMaxNewton);
  C.nc_cap = nc;
}

// Buffers and expansion maps of a step with n_contacts = nc when pairs are
// set: contacts 0..P-1 are the pairs (their slots, indices into the pairs'
// distinct nodes), contacts P..nc-1 the obstacle contacts (one slot each,
// the node after the pairs' nodes in the build's list).
void ensure_pair_step(icr_scene *s, int nc) {
  auto &Pr = s->pairs;
  if (Pr.count == 0 || Pr.step_nc == nc) return;
  ICR_HIP(hipStreamSynchronize(s->stream));
  s->epoch++;
  Pr.step_arena.release();
  const int P = Pr.count, nu = Pr.nu + nc - P;
  std::vector<int> idx(4L * nc, -1);
  std::vector<double> w(4L * nc, 0.0);
  for (long e = 0; e < 4L * P; ++e) {
    idx[e] = Pr.idx[e];
    w[e] = Pr.w[e];
  }
  for (int c = P; c < nc; ++c) {
    idx[4L * c] = Pr.nu + c - P;
    w[4L * c] = 1.0;
  }
  auto &A = Pr.step_arena;
  Pr.d_unodes = A.alloc<int>(nu);
  Pr.d_idx = A.upload(idx, s->stream);
  Pr.d_wexp = A.upload(w, s->stream);
  Pr.d_WN = A.alloc<double>(9L * nu * nu);
  Pr.d_fu = A.alloc<double>(3L * nu);
  ICR_HIP(hipStreamSynchronize(s->stream));
  Pr.step_nc = nc;
}

// Host-side build of the factor descriptors from the symbolic structure.
void prepare_factor(icr_scene *s) {
  auto &m = s->mesh;
  auto &F = s->fac;
  const auto &g = m.graph;
  analyze(m.nodes.data(), g, 48, F.sym);
  std::string bad = check_symbolic(g, F.sym);
  if (!bad.empty()) throw std::runtime_error("symbolic analysis: " + bad);
  const Symbolic &sym = F.sym;
  const int ns = sym.nsup;
  F.sup.assign(ns, SupDev{});
  long long fo = 0, lo = 0, xo = 0;
  F.nnzL = 0;
  F.flops = 0;
  F.max_front = 0;
  for (int s_ = 0; s_ < ns; ++s_) {
    SupDev &d = F.sup[s_];
    d.col0 = sym.col0[s_];
    d.ncol = sym.ncol[s_];
    d.nb = sym.rows_ptr[s_ + 1] - sym.rows_ptr[s_];
    d.parent = sym.parent[s_];
    d.rows_off = sym.rows_ptr[s_];
    d.first_desc = sym.first_desc[s_];
    d.child_off = sym.child_ptr[s_];
    d.nchild = sym.child_ptr[s_ + 1] - sym.child_ptr[s_];
    d.region_nodes = sym.col0[s_] + sym.ncol[s_] - sym.col0[sym.first_desc[s_]];
    const long long f = 3LL * (d.ncol + d.nb), n3 = 3LL * d.ncol;
    d.front_off = fo;
    d.linv_off = lo;
    d.x1_off = xo;
    fo += f * f;
    lo += n3 * n3;
    xo += f;
    F.nnzL += n3 * (n3 + 1) / 2 + (f - n3) * n3;
    for (long long c = 0; c < n3; ++c) F.flops += (double)(f - c) * (double)(f - c);
    F.max_front = std::max<int>(F.max_front, (int)f);
  }
  F.front_elems = fo;
  F.linv_elems = lo;
  F.x1_elems = xo;
  // child index maps (parent local node -> child below-row index, or -1)
  std::vector<int> invmap_off(sym.child.size()), invmap;
  for (int p = 0; p < ns; ++p) {
    const SupDev &P = F.sup[p];
    const int np = P.ncol + P.nb;
    for (int e = sym.child_ptr[p]; e < sym.child_ptr[p + 1]; ++e) {
      const int c = sym.child[e];
      invmap_off[e] = (int)invmap.size();
      invmap.resize(invmap.size() + np, -1);
      int *inv = invmap.data() + invmap_off[e];
      for (int i = sym.rows_ptr[c]; i < sym.rows_ptr[c + 1]; ++i) {
        int r = sym.rows[i];
        int L;
        if (r >= P.col0 && r < P.col0 + P.ncol)
          L = r - P.col0;
        else {
          auto it = std::lower_bound(sym.rows.begin() + sym.rows_ptr[p], sym.rows.begin() + sym.rows_ptr[p + 1], r);
          L = P.ncol + (int)(it - (sym.rows.begin() + sym.rows_ptr[p]));
        }
        inv[L] = i - sym.rows_ptr[c];
      }
    }
  }
  // A -> front scatter entries, grouped by level
  std::vector<std::vector<AScatter>> per_level(sym.nlevels);
  std::vector<int> bsr_ptr(g.ptr.begin(), g.ptr.end());
  for (int s_ = 0; s_ < ns; ++s_) {
    const SupDev &S = F.sup[s_];
    for (int p = S.col0; p < S.col0 + S.ncol; ++p) {
      const int v = sym.perm[p];
      for (int e = g.ptr[v]; e < g.ptr[v + 1]; ++e) {
        const int u = g.adj[e];
        const int q = sym.iperm[u];
        if (q < p) continue;
        int lr;
        if (q < S.col0 + S.ncol)
          lr = q - S.col0;
        else {
          auto it = std::lower_bound(sym.rows.begin() + S.rows_off, sym.rows.begin() + S.rows_off + S.nb, q);
          if (it == sym.rows.begin() + S.rows_off + S.nb || *it != q)
            throw std::runtime_error("A entry outside the supernodal structure");
          lr = S.ncol + (int)(it - (sym.rows.begin() + S.rows_off));
        }
        // block (row u, col v) of the BSR matrix
        auto jt = std::lower_bound(g.adj.begin() + g.ptr[u], g.adj.begin() + g.ptr[u + 1], v);
        int blk = (int)(jt - g.adj.begin());
        per_level[sym.height[s_]].push_back(AScatter{s_, lr, p - S.col0, blk});
      }
    }
  }
  std::vector<AScatter> ascat;
  F.levels.assign(sym.nlevels, LevelInfo{});
  for (int l = 0; l < sym.nlevels; ++l) {
    LevelInfo &L = F.levels[l];
    L.first = sym.level_ptr[l];
    L.count = sym.level_ptr[l + 1] - sym.level_ptr[l];
    L.a_first = (int)ascat.size();
    L.a_count = (int)per_level[l].size();
    ascat.insert(ascat.end(), per_level[l].begin(), per_level[l].end());
    for (int q = L.first; q < L.first + L.count; ++q) {
      const SupDev &S = F.sup[sym.level_sup[q]];
      int n3 = 3 * S.ncol, b3 = 3 * S.nb, f = n3 + b3;
      L.max_n3 = std::max(L.max_n3, n3);
      L.max_f3 = std::max(L.max_f3, f);
      L.max_b3 = std::max(L.max_b3, b3);
      L.max_f2 = std::max<long long>(L.max_f2, (long long)f * f);
      L.max_rows_tiles = std::max(L.max_rows_tiles, cdiv(n3, TILE));
      L.max_below_tiles = std::max(L.max_below_tiles, cdiv(b3, TILE));
    }
  }
  // single-RHS task lists: every (supernode, block) of a level that exists;
  // k-chunks of the forward products: a level with fewer than 256 row blocks
  // of 64 splits each block's k range (of at least 256 per chunk) over up to
  // 16 blocks
  std::vector<int2> srhs;
  long long fwd_part = 0;
  for (LevelInfo &L : F.levels) {
    const int rows_of[3] = {64, 64, 16};
    for (int k = 0; k < 3; ++k) {
      L.srhs_off[k] = (int)srhs.size();
      for (int q = 0; q < L.count; ++q) {
        const SupDev &S = F.sup[sym.level_sup[L.first + q]];
        const int len = (k == SR_FWD_OFF) ? 3 * S.nb : 3 * S.ncol;
        for (int bk = 0; bk < cdiv(len, rows_of[k]); ++bk) srhs.push_back(make_int2(q, bk));
      }
      L.srhs_cnt[k] = (int)srhs.size() - L.srhs_off[k];
    }
    auto split = [&](int blocks, int k) {
      if (blocks <= 0 || blocks >= 256) return 1;
      return std::max(1, std::min({16, cdiv(512, blocks), k / 256}));
    };
    L.fwd_split_diag = split(L.srhs_cnt[SR_FWD_DIAG], L.max_n3);
    L.fwd_split_off = split(L.srhs_cnt[SR_FWD_OFF], L.max_n3);
    fwd_part = std::max({fwd_part, (long long)L.srhs_cnt[SR_FWD_DIAG] * L.fwd_split_diag,
                         (long long)L.srhs_cnt[SR_FWD_OFF] * L.fwd_split_off});
  }
  std::vector<int> sup_of_node(m.N);
  for (int s_ = 0; s_ < ns; ++s_)
    for (int p = sym.col0[s_]; p < sym.col0[s_] + sym.ncol[s_]; ++p) sup_of_node[sym.perm[p]] = s_;

  s->fac_arena.release();
  F.rhs_arena.release();
  F.nc_cap = 0;
  F.fac32_arena.release();
  F.have32 = false;
  F.mixed_arena.release();
  F.mixed_cap = 0;
  hipStream_t st = s->stream;
  auto &A = s->fac_arena;
  F.d_sup = A.upload(F.sup, st);
  F.d_rows = A.upload(sym.rows, st);
  F.d_child = A.upload(sym.child, st);
  F.d_invmap_off = A.upload(invmap_off, st);
  F.d_invmap = A.upload(invmap, st);
  F.d_level_sup = A.upload(sym.level_sup, st);
  F.d_perm = A.upload(sym.perm, st);
  F.d_iperm = A.upload(sym.iperm, st);
  F.d_sup_of_node = A.upload(sup_of_node, st);
  F.d_ascat = A.upload(ascat, st);
  F.d_front = A.alloc<double>(F.front_elems);
  F.d_linv = A.alloc<double>(F.linv_elems);
  F.d_x1 = A.alloc<double>(F.x1_elems);
  F.d_y = A.alloc<double>(2L * m.n);
  F.d_err = A.alloc<int>(1);
  F.d_fwd_part = A.alloc<double>(std::max(1LL, fwd_part * 64));
  F.d_srhs_tasks = A.upload(srhs, st);
  ICR_HIP(hipStreamSynchronize(st));
}

void check_obstacle(const icr_obstacle *o) {
  REQUIRE(o != nullptr, "obstacle is NULL");
  REQUIRE(o->kind == 0 || o->kind == 1, "obstacle kind must be 0 (plane) or 1 (sphere)");
  if (o->kind == 1) REQUIRE(std::isfinite(o->radius) && o->radius > 0, "sphere radius must be positive");
  if (o->kind == 0) {
    double n2 = o->normal[0] * o->normal[0] + o->normal[1] * o->normal[1] + o->normal[2] * o->normal[2];
    REQUIRE(std::fabs(n2 - 1.0) < 1e-12, "plane normal must be a unit vector");
  }
}

}  // namespace

extern "C" {

icr_status icr_create(icr_scene **out, void *stream) {
  if (!out) return ICR_E_ARG;
  *out = nullptr;
  icr_scene *s = new (std::nothrow) icr_scene();
  if (!s) return ICR_E_OOM;
  s->stream = (hipStream_t)stream;
  if (hipInit(0) != hipSuccess || hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return ICR_E_HIP;
  }
  if (hipDeviceGetAttribute(&s->clock_khz, hipDeviceAttributeWallClockRate, s->device) != hipSuccess)
    s->clock_khz = 0;
  *out = s;
  return ICR_OK;
}

void icr_destroy(icr_scene *s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->stream);
  if (s->side) (void)hipStreamSynchronize(s->side);
  s->sg.reset();
  if (s->sg.cap) (void)hipStreamDestroy(s->sg.cap);
  if (s->ev_fork) (void)hipEventDestroy(s->ev_fork);
  if (s->ev_join) (void)hipEventDestroy(s->ev_join);
  if (s->side) (void)hipStreamDestroy(s->side);
  s->con.arena.release();
  s->map_arena.release();
  s->pairs.arena.release();
  s->pairs.step_arena.release();
  s->fac.rhs_arena.release();
  s->fac.fac32_arena.release();
  s->fac.mixed_arena.release();
  s->fac_arena.release();
  s->mesh_arena.release();
  s->state_arena.release();
  delete s;
}

const char *icr_last_error(const icr_scene *s) { return s ? s->err.c_str() : "null scene"; }

icr_status icr_set_stream(icr_scene *s, void *stream) {
  return guarded(s, [&] {
    s->stream = (hipStream_t)stream;
    return ICR_OK;
  });
}

icr_status icr_set_overlap(icr_scene *s, int32_t enable) {
  return guarded(s, [&] {
    REQUIRE(enable == 0 || enable == 1, "enable must be 0 or 1");
    if (s->overlap != (enable == 1)) {
      s->overlap = enable == 1;
      s->epoch++;   // a captured step graph holds the other launch pattern
    }
    return ICR_OK;
  });
}

icr_status icr_assemble(icr_scene *s, const double *nodes, int32_t N, const int32_t *tets, int32_t T,
                        const double *E, const double *nu, double rho, double alpha, double beta, double h,
                        const double *gravity, const uint8_t *fixed) {
  return guarded(s, [&] {
    REQUIRE(nodes && tets && E && nu && gravity && fixed, "NULL host array");
    REQUIRE(N > 0 && T > 0, "N and T must be positive");
    REQUIRE(N < (1 << 24), "at most 2^24 - 1 nodes");
    REQUIRE(std::isfinite(h) && h > 0, "h must be positive and finite");
    REQUIRE(rho > 0 && alpha >= 0 && beta >= 0, "rho > 0, alpha >= 0, beta >= 0 required");
    for (long i = 0; i < 4L * T; ++i) REQUIRE(tets[i] >= 0 && tets[i] < N, "tet references a node out of range");
    for (int t = 0; t < T; ++t) {
      REQUIRE(std::isfinite(E[t]) && E[t] > 0, "E must be positive");
      REQUIRE(nu[t] > 0 && nu[t] < 0.5, "nu must be in (0, 0.5)");
    }
    ICR_HIP(hipStreamSynchronize(s->stream));
    s->epoch++;
    s->sg.reset();
    s->assembled = s->factored = s->has_candidates = s->stepped = false;
    s->con.arena.release();
    s->con.nc_cap = 0;
    s->map_arena.release();
    s->map_nc_cap = s->map_nu_cap = 0;
    s->pairs.arena.release();
    s->pairs.step_arena.release();
    s->pairs = Pairs();
    s->fac.rhs_arena.release();
    s->fac.nc_cap = 0;
    s->fac.fac32_arena.release();
    s->fac.have32 = false;
    s->fac.mixed_arena.release();
    s->fac.mixed_cap = 0;
    s->fac_arena.release();
    s->mesh_arena.release();
    s->state_arena.release();
    auto &m = s->mesh;
    m.N = N;
    m.T = T;
    m.n = 3 * N;
    m.rho = rho;
    m.alpha = alpha;
    m.beta = beta;
    m.h = h;
    for (int a = 0; a < 3; ++a) m.grav[a] = gravity[a];
    m.nodes.assign(nodes, nodes + 3L * N);
    m.tets.assign(tets, tets + 4L * T);
    m.fixed.assign(fixed, fixed + N);
    m.graph = build_graph(N, tets, T);
    const auto &g = m.graph;
    m.nnzb = g.ptr[N];
    std::vector<int> bsr_row(m.nnzb);
    for (int i = 0; i < N; ++i)
      for (int e = g.ptr[i]; e < g.ptr[i + 1]; ++e) bsr_row[e] = i;
    // element contributions per block, ascending element order
    std::vector<int> cnt(m.nnzb + 1, 0), nt_cnt(N + 1, 0);
    auto block_of = [&](int u, int v) {
      auto it = std::lower_bound(g.adj.begin() + g.ptr[u], g.adj.begin() + g.ptr[u + 1], v);
      return (int)(it - g.adj.begin());
    };
    for (int t = 0; t < T; ++t)
      for (int a = 0; a < 4; ++a) {
        nt_cnt[tets[4 * t + a] + 1]++;
        for (int b = 0; b < 4; ++b) cnt[block_of(tets[4 * t + a], tets[4 * t + b]) + 1]++;
      }
    for (int i = 0; i < m.nnzb; ++i) cnt[i + 1] += cnt[i];
    for (int i = 0; i < N; ++i) nt_cnt[i + 1] += nt_cnt[i];
    std::vector<int> contrib(cnt[m.nnzb]), fillp(cnt.begin(), cnt.end() - 1);
    std::vector<int> nt(nt_cnt[N]), filln(nt_cnt.begin(), nt_cnt.end() - 1);
    for (int t = 0; t < T; ++t)
      for (int a = 0; a < 4; ++a) {
        nt[filln[tets[4 * t + a]]++] = t;
        for (int b = 0; b < 4; ++b) contrib[fillp[block_of(tets[4 * t + a], tets[4 * t + b])]++] = t * 16 + a * 4 + b;
      }
    hipStream_t st = s->stream;
    auto &A = s->mesh_arena;
    m.d_nodes = A.upload(m.nodes, st);
    m.d_tets = A.upload(m.tets, st);
    m.d_E = A.upload(std::vector<double>(E, E + T), st);
    m.d_nu = A.upload(std::vector<double>(nu, nu + T), st);
    m.d_fixed = A.upload(m.fixed, st);
    m.d_bsr_ptr = A.upload(g.ptr, st);
    m.d_bsr_col = A.upload(g.adj, st);
    m.d_bsr_row = A.upload(bsr_row, st);
    m.d_contrib_ptr = A.upload(cnt, st);
    m.d_contrib = A.upload(contrib, st);
    m.d_nt_ptr = A.upload(nt_cnt, st);
    m.d_nt = A.upload(nt, st);
    m.d_Ke = A.alloc<double>(144L * T);
    m.d_vol = A.alloc<double>(T);
    m.d_mass = A.alloc<double>(N);
    m.d_K = A.alloc<double>(9L * m.nnzb);
    m.d_A = A.alloc<double>(9L * m.nnzb);
    m.d_err = A.alloc<int>(1);
    ICR_HIP(hipMemsetAsync(m.d_err, 0x7f, sizeof(int), st));
    launch_element_matrices(s);
    launch_assemble_blocks(s);
    int bad = 0;
    ICR_HIP(hipMemcpyAsync(&bad, m.d_err, sizeof(int), hipMemcpyDeviceToHost, st));
    ICR_HIP(hipStreamSynchronize(st));
    if (bad != 0x7f7f7f7f) throw ArgError("tetrahedron " + std::to_string(bad) + " has non-positive volume");
    // state
    auto &S = s->st;
    auto &B = s->state_arena;
    S.d_q = B.upload(m.nodes, st);
    S.d_qrest = B.upload(m.nodes, st);
    S.d_v = B.alloc<double>(m.n);
    ICR_HIP(hipMemsetAsync(S.d_v, 0, sizeof(double) * m.n, st));
    S.d_b = B.alloc<double>(m.n);
    S.d_dvfree = B.alloc<double>(m.n);
    S.d_qfree = B.alloc<double>(m.n);
    S.d_sol = B.alloc<double>(m.n);
    S.d_node_force = B.alloc<double>(m.n);
    ICR_HIP(hipMemsetAsync(S.d_node_force, 0, sizeof(double) * m.n, st));
    S.d_prev_nodes = B.alloc<int>(N);
    S.d_prev_nc = B.alloc<int>(1);
    ICR_HIP(hipMemsetAsync(S.d_prev_nc, 0, sizeof(int), st));
    S.t = 0;
    S.d_ctx = B.alloc<StepCtx>(1);
    S.d_stamps = B.alloc<unsigned long long>(6 + 4 * kMaxNewton);
    S.obs_valid = false;
    {
      double t0 = 0.0;
      launch_set_ctx(s, nullptr, &t0);
    }
    ICR_HIP(hipStreamSynchronize(st));
    s->assembled = true;
    return ICR_OK;
  });
}

icr_status icr_factor(icr_scene *s) {
  return guarded(s, [&] {
    if (!s->assembled) throw StateError("icr_factor before icr_assemble");
    s->factored = false;
    s->epoch++;
    prepare_factor(s);
    run_numeric_factor(s);
    int bad = 0;
    ICR_HIP(hipMemcpy(&bad, s->fac.d_err, sizeof(int), hipMemcpyDeviceToHost));
    if (bad != 0x7f7f7f7f)
      throw SpdError("non-positive pivot at permuted column " + std::to_string(bad));
    s->factored = true;
    return ICR_OK;
  });
}

icr_status icr_get_factor_info(icr_scene *s, icr_factor_info *out) {
  return guarded(s, [&] {
    REQUIRE(out, "NULL output");
    if (!s->factored) throw StateError("no factor");
    out->n = s->mesh.n;
    out->n_supernodes = s->fac.sym.nsup;
    out->n_levels = s->fac.sym.nlevels;
    out->nnz_L = s->fac.nnzL;
    out->max_front = s->fac.max_front;
    out->factor_flops = s->fac.flops;
    out->factor_ms = s->fac.ms;
    out->device_bytes = (int64_t)(s->mesh_arena.bytes + s->fac_arena.bytes + s->fac.rhs_arena.bytes +
                                  s->state_arena.bytes + s->con.arena.bytes + s->map_arena.bytes +
                                  s->fac.fac32_arena.bytes + s->fac.mixed_arena.bytes + s->pairs.arena.bytes +
                                  s->pairs.step_arena.bytes);
    return ICR_OK;
  });
}

icr_status icr_build_WH(icr_scene *s, int32_t n_c, const int32_t *node_ids, const double *weights, double *WH) {
  return guarded(s, [&] {
    if (!s->factored) throw StateError("icr_build_WH before icr_factor");
    REQUIRE(n_c >= 1 && n_c <= 8192, "n_c must be in [1, 8192]");
    REQUIRE(node_ids && WH, "NULL device pointer");
    hipStream_t st = s->stream;
    auto device_check = [&] {
      int bad = 0;
      ICR_HIP(hipMemcpyAsync(&bad, s->fac.d_cerr, sizeof(int), hipMemcpyDeviceToHost, st));
      ICR_HIP(hipStreamSynchronize(st));
      if (bad == 1) throw ArgError("a contact node id is out of range or clamped");
      if (bad) throw ArgError("duplicate contact node ids");
    };
    if (!weights) {   // nodal contacts
      REQUIRE(n_c <= s->mesh.N, "more contacts than nodes");
      ensure_rhs_capacity(s, n_c);
      build_WH_device(s, n_c, node_ids, WH, true);
      device_check();
      return ICR_OK;
    }
    // mapped contacts: W_N of the distinct nodes, then the weighted expansion
    std::vector<int> ids(4L * n_c);
    std::vector<double> w(4L * n_c);
    ICR_HIP(hipMemcpyAsync(ids.data(), node_ids, sizeof(int) * ids.size(), hipMemcpyDeviceToHost, st));
    ICR_HIP(hipMemcpyAsync(w.data(), weights, sizeof(double) * w.size(), hipMemcpyDeviceToHost, st));
    ICR_HIP(hipStreamSynchronize(st));
    const auto &mesh = s->mesh;
    std::vector<int> nodes;
    nodes.reserve(ids.size());
    for (int c = 0; c < n_c; ++c) {
      int used = 0;
      for (int k = 0; k < 4; ++k) {
        const int v = ids[4 * c + k];
        if (v == -1) continue;
        REQUIRE(v >= 0 && v < mesh.N, "contact " + std::to_string(c) + ": node id out of range");
        REQUIRE(!mesh.fixed[v], "contact " + std::to_string(c) + ": node is clamped");
        REQUIRE(std::isfinite(w[4 * c + k]) && w[4 * c + k] != 0.0,
                "contact " + std::to_string(c) + ": weights of used slots must be finite and non-zero");
        for (int l = 0; l < k; ++l) REQUIRE(ids[4 * c + l] != v, "contact " + std::to_string(c) + ": repeated node");
        nodes.push_back(v);
        ++used;
      }
      REQUIRE(used > 0, "contact " + std::to_string(c) + " has no node");
    }
    std::sort(nodes.begin(), nodes.end());
    nodes.erase(std::unique(nodes.begin(), nodes.end()), nodes.end());
    const int nu = (int)nodes.size();
    REQUIRE(nu <= 8192, "the contacts reference more than 8192 distinct nodes");
    std::vector<int> idx(4L * n_c, -1);
    for (long e = 0; e < 4L * n_c; ++e)
      if (ids[e] >= 0) idx[e] = (int)(std::lower_bound(nodes.begin(), nodes.end(), ids[e]) - nodes.begin());
    if (n_c > s->map_nc_cap || nu > s->map_nu_cap) {
      ICR_HIP(hipStreamSynchronize(st));
      s->map_arena.release();
      s->map_nc_cap = std::max(n_c, s->map_nc_cap);
      s->map_nu_cap = std::max(nu, s->map_nu_cap);
      s->d_map_nodes = s->map_arena.alloc<int>(s->map_nu_cap);
      s->d_map_idx = s->map_arena.alloc<int>(4L * s->map_nc_cap);
      s->d_map_WN = s->map_arena.alloc<double>(9L * s->map_nu_cap * s->map_nu_cap);
    }
    ICR_HIP(hipMemcpyAsync(s->d_map_nodes, nodes.data(), sizeof(int) * nu, hipMemcpyHostToDevice, st));
    ICR_HIP(hipMemcpyAsync(s->d_map_idx, idx.data(), sizeof(int) * idx.size(), hipMemcpyHostToDevice, st));
    ensure_rhs_capacity(s, nu);
    build_WH_device(s, nu, s->d_map_nodes, s->d_map_WN, true);
    launch_wh_expand(st, n_c, nu, s->d_map_idx, weights, s->d_map_WN, WH);
    device_check();   // also keeps the host arrays alive until the copies are done
    return ICR_OK;
  });
}

icr_status icr_update_W(icr_scene *s, int32_t n_c, const double *WH, const double *C, double *W) {
  return guarded(s, [&] {
    REQUIRE(n_c >= 1, "n_c must be >= 1");
    REQUIRE(WH && C && W, "NULL device pointer");
    REQUIRE(W != WH, "W may not alias WH");
    launch_update_W<double>(s->stream, n_c, WH, C, W);
    return ICR_OK;
  });
}

icr_status icr_solve_contacts(icr_scene *s, int32_t n_c, const double *W, const double *d, const double *mu,
                              double h, double *lambda, int8_t *status, int32_t max_sweeps, double tol,
                              int32_t j_inner, int32_t *sweeps_out, double *eps_out) {
  return guarded(s, [&] {
    REQUIRE(n_c >= 1 && n_c <= kPgsMaxContacts, "n_c must be in [1, 4096]");
    REQUIRE(max_sweeps >= 1, "max_sweeps must be >= 1");
    REQUIRE(j_inner >= 0, "j_inner must be >= 0");
    REQUIRE(std::isfinite(h) && h > 0, "h must be positive");
    REQUIRE(W && d && mu && lambda && status, "NULL device pointer");
    ensure_contact_buffers(s, std::max(n_c, 1));
    launch_pgs<double>(s->stream, n_c, W, d, mu, h, lambda, status, max_sweeps, tol, j_inner, s->con.d_sweeps,
               s->con.d_eps, s->con.pgs);
    if (sweeps_out || eps_out) {
      int sw = 0;
      double ep = 0;
      ICR_HIP(hipMemcpyAsync(&sw, s->con.d_sweeps, sizeof(int), hipMemcpyDeviceToHost, s->stream));
      ICR_HIP(hipMemcpyAsync(&ep, s->con.d_eps, sizeof(double), hipMemcpyDeviceToHost, s->stream));
      ICR_HIP(hipStreamSynchronize(s->stream));
      if (sweeps_out) *sweeps_out = sw;
      if (eps_out) *eps_out = ep;
      if (!(ep <= tol)) return ICR_WARN_NOT_CONVERGED;
    }
    return ICR_OK;
  });
}

icr_status icr_proximity_update(icr_scene *s, int32_t n_c, const double *WH, const double *p_free, const double *f,
                                double h, double *p) {
  return guarded(s, [&] {
    REQUIRE(n_c >= 1, "n_c must be >= 1");
    REQUIRE(std::isfinite(h) && h > 0, "h must be positive");
    REQUIRE(WH && p_free && f && p, "NULL device pointer");
    launch_proximity<double>(s->stream, n_c, WH, p_free, f, h, p);
    return ICR_OK;
  });
}

icr_status icr_set_pairs(icr_scene *s, int32_t count, const int32_t *node_ids, const double *weights,
                         const double *normals, const double *mu) {
  return guarded(s, [&] {
    if (!s->assembled) throw StateError("icr_set_pairs before icr_assemble");
    REQUIRE(count >= 0 && count <= kPgsMaxContacts, "pair count must be in [0, 4096]");
    REQUIRE(count == 0 || (node_ids && weights && normals && mu), "NULL host array");
    const auto &mesh = s->mesh;
    std::vector<int> nodes;
    for (int c = 0; c < count; ++c) {
      int used = 0;
      const std::string who = "pair " + std::to_string(c);
      for (int k = 0; k < 4; ++k) {
        const int v = node_ids[4 * c + k];
        if (v == -1) continue;
        REQUIRE(v >= 0 && v < mesh.N, who + ": node id out of range");
        REQUIRE(!mesh.fixed[v], who + ": node is clamped");
        REQUIRE(std::isfinite(weights[4 * c + k]) && weights[4 * c + k] != 0.0,
                who + ": weights of used slots must be finite and non-zero");
        for (int l = 0; l < k; ++l) REQUIRE(node_ids[4 * c + l] != v, who + ": repeated node");
        nodes.push_back(v);
        ++used;
      }
      REQUIRE(used > 0, who + " has no node");
      const double *n = normals + 3 * c;
      REQUIRE(std::fabs(n[0] * n[0] + n[1] * n[1] + n[2] * n[2] - 1.0) < 1e-12, who + ": normal must be a unit vector");
      REQUIRE(std::isfinite(mu[c]) && mu[c] >= 0, who + ": friction must be >= 0");
    }
    std::sort(nodes.begin(), nodes.end());
    nodes.erase(std::unique(nodes.begin(), nodes.end()), nodes.end());
    REQUIRE((int)nodes.size() <= 8192, "the pairs reference more than 8192 distinct nodes");
    for (int v : s->con.nodes)
      REQUIRE(!std::binary_search(nodes.begin(), nodes.end(), v), "a pair node is a contact candidate");
    ICR_HIP(hipStreamSynchronize(s->stream));
    s->epoch++;
    auto &Pr = s->pairs;
    Pr.arena.release();
    Pr.step_arena.release();
    Pr = Pairs();
    if (count == 0) return ICR_OK;
    Pr.count = count;
    Pr.nodes = nodes;
    Pr.nu = (int)nodes.size();
    Pr.idx.assign(4L * count, -1);
    Pr.w.assign(4L * count, 0.0);
    std::vector<int> slot_node(4L * count, -1), cnt(Pr.nu + 1, 0);
    for (long e = 0; e < 4L * count; ++e) {
      if (node_ids[e] < 0) continue;
      slot_node[e] = node_ids[e];
      Pr.idx[e] = (int)(std::lower_bound(nodes.begin(), nodes.end(), node_ids[e]) - nodes.begin());
      Pr.w[e] = weights[e];
      cnt[Pr.idx[e] + 1]++;
    }
    for (int u = 0; u < Pr.nu; ++u) cnt[u + 1] += cnt[u];
    std::vector<int> csr(cnt[Pr.nu]), fill(cnt.begin(), cnt.end() - 1);
    for (long e = 0; e < 4L * count; ++e)
      if (Pr.idx[e] >= 0) csr[fill[Pr.idx[e]]++] = (int)e;   // ascending slot order per node
    hipStream_t st = s->stream;
    auto &A = Pr.arena;
    Pr.d_slot_node = A.upload(slot_node, st);
    Pr.d_w = A.upload(Pr.w, st);
    Pr.d_normal = A.upload(std::vector<double>(normals, normals + 3L * count), st);
    Pr.d_mu = A.upload(std::vector<double>(mu, mu + count), st);
    Pr.d_force = A.alloc<double>(3L * count);
    ICR_HIP(hipMemsetAsync(Pr.d_force, 0, sizeof(double) * 3 * count, st));
    Pr.d_nodes = A.upload(nodes, st);
    Pr.d_csr_ptr = A.upload(cnt, st);
    Pr.d_csr_slot = A.upload(csr, st);
    ICR_HIP(hipStreamSynchronize(st));
    return ICR_OK;
  });
}

icr_status icr_set_candidates(icr_scene *s, int32_t count, const int32_t *nodes, const double *mu) {
  return guarded(s, [&] {
    if (!s->assembled) throw StateError("icr_set_candidates before icr_assemble");
    REQUIRE(count >= 1 && count <= 4096, "candidate count must be in [1, 4096]");
    REQUIRE(nodes && mu, "NULL host array");
    std::vector<double> mu_node(s->mesh.n / 3, 0.0);
    std::vector<uint8_t> seen(s->mesh.N, 0);
    for (int i = 0; i < count; ++i) {
      int v = nodes[i];
      REQUIRE(v >= 0 && v < s->mesh.N, "candidate node out of range");
      REQUIRE(!s->mesh.fixed[v], "candidate node is clamped");
      REQUIRE(!seen[v]++, "duplicate candidate node");
      REQUIRE(!std::binary_search(s->pairs.nodes.begin(), s->pairs.nodes.end(), v),
              "candidate node belongs to a pair contact");
      REQUIRE(std::isfinite(mu[i]) && mu[i] >= 0, "friction must be >= 0");
      mu_node[v] = mu[i];
    }
    auto &C = s->con;
    C.count = count;
    // ascending node id: the selection kernel places its contacts in list order
    C.nodes.assign(nodes, nodes + count);
    std::sort(C.nodes.begin(), C.nodes.end());
    auto &B = s->state_arena;
    s->epoch++;
    C.d_cand = B.upload(C.nodes, s->stream);
    C.d_mu_node = B.upload(mu_node, s->stream);
    ICR_HIP(hipStreamSynchronize(s->stream));
    s->has_candidates = true;
    return ICR_OK;
  });
}

namespace {

// Preconditions of icr_step (throws the error icr_step returns).
void check_step(icr_scene *s, const icr_obstacle *obs, const icr_step_opts *opt) {
  if (!s->factored) throw StateError("icr_step before icr_factor");
  if (!s->has_candidates) throw StateError("icr_step before icr_set_candidates");
  check_obstacle(obs);
  REQUIRE(opt, "NULL options");
  const int nc = opt->n_contacts;
  const int P = s->pairs.count;
  REQUIRE(nc >= 1 && nc >= P && nc - P <= s->con.count,
          "n_contacts must be in [1, pair count + candidate count] and at least the pair count");
  REQUIRE(P == 0 || opt->scheme == 0, "pair contacts run in the fast scheme (scheme 0) only");
  REQUIRE(P == 0 || s->pairs.nu + nc - P <= 8192, "pair nodes and obstacle contacts exceed 8192 nodes");
  REQUIRE(nc <= kPgsMaxContacts, "n_contacts exceeds the PGS kernel limit (4096)");
  REQUIRE(opt->n_newton >= 1 && opt->n_newton <= kMaxNewton, "n_newton must be in [1, 256]");
  REQUIRE(opt->max_sweeps >= 1 && opt->j_inner >= 0, "max_sweeps >= 1 and j_inner >= 0 required");
  REQUIRE(opt->scheme >= 0 && opt->scheme <= 2, "scheme must be 0 (fast), 1 (standard) or 2 (per constraint)");
  REQUIRE(opt->graph == 0 || opt->graph == 1, "graph must be 0 or 1");
  REQUIRE(opt->precision == ICR_FP64 || opt->precision == ICR_FP32_IR, "precision must be ICR_FP64 or ICR_FP32_IR");
  REQUIRE(opt->precision == ICR_FP64 || opt->scheme == 0, "ICR_FP32_IR runs the fast scheme (scheme 0) only");
  REQUIRE(opt->refine >= 0 && opt->refine <= 2, "refine must be in [0, 2]");
}

// Enqueue one whole time step on s->stream.  With opt->timing, one-thread
// kernels stamp the device clock between phases (slots 0..5 for the step,
// 6 + 4k + j for Newton iteration k); stamps work the same in a replayed
// graph.  Every argument that changes from step to step lives in device
// memory, so the sequence can be captured once and replayed.
constexpr int kStampStep = 0, kStampNewton = 6;   // phase stamps of a timed step

// The step up to its Newton loop: free motion, contacts, W_H (Algorithm 3
// before step 1).
void enqueue_pre(icr_scene *s, const icr_step_opts *opt) {
  hipStream_t st = s->stream;
  auto &C = s->con;
  auto &S = s->st;
  const int nc = opt->n_contacts;
  const bool standard = opt->scheme == 1;
  auto mark = [&](int base, int i) {
    if (opt->timing) launch_stamp(s, base + i);
  };
  const int ev = kStampStep;
  mark(ev, 0);
  // free motion (Eq. 5, 12)
  launch_free_rhs(s, S.d_q, S.d_v, S.d_b);
  single_rhs_solve(s, S.d_b, S.d_dvfree);
  launch_axpy_qfree(s);
  mark(ev, 1);
  auto &Pr = s->pairs;
  const int P = Pr.count;
  if (nc > P) launch_select_contacts(s, nc);
  if (P > 0) launch_pair_points(s, nc);   // and the node list of the W_H build
  mark(ev, 2);
  const bool mixed = opt->precision == ICR_FP32_IR;
  if (P > 0) {
    // pairs: nodal W_N of the distinct nodes, then W_H = H_w W_N H_w^T
    const int nu = Pr.nu + nc - P;
    if (mixed)
      build_WH_mixed(s, nu, Pr.d_unodes, opt->refine, nullptr, Pr.d_WN);
    else
      build_WH_device(s, nu, Pr.d_unodes, Pr.d_WN, false);
    launch_wh_expand(st, nc, nu, Pr.d_idx, Pr.d_wexp, Pr.d_WN, C.d_WH);
    if (mixed) launch_narrow(s, C.d_WH, C.d_WH32, 9L * nc * nc);
  } else if (mixed) {
    build_WH_mixed(s, nc, C.d_nodes_c, opt->refine, C.d_WH32, nullptr);
  } else if (!standard) {
    build_WH_device(s, nc, C.d_nodes_c, C.d_WH, false);
  }
  mark(ev, 3);
}

// Algorithm 3's Newton loop (steps 1-4), or its variants.
void enqueue_newton(icr_scene *s, const icr_step_opts *opt) {
  hipStream_t st = s->stream;
  auto &C = s->con;
  auto &S = s->st;
  const double h = s->mesh.h;
  const int nc = opt->n_contacts, nk = opt->n_newton;
  const bool standard = opt->scheme == 1;
  const bool per_constraint = opt->scheme == 2;
  const bool mixed = opt->precision == ICR_FP32_IR;
  auto mark = [&](int base, int i) {
    if (opt->timing) launch_stamp(s, base + i);
  };
  const int kev = kStampNewton;
  // directions updated before every local solve: proximity of the warm start
  if (per_constraint) launch_proximity<double>(st, nc, C.d_WH, C.d_pfree, C.d_f, h, C.d_p);
  for (int k = 0; k < nk; ++k) {
    if (per_constraint) {
      mark(kev, 4 * k);
      mark(kev, 4 * k + 1);
      launch_pgs_per_constraint(st, nc, S.d_ctx, C.d_WH, C.d_pfree, C.d_p, C.d_pstart, C.d_mu, h, C.d_f, C.d_C,
                                C.d_lam, C.d_status, opt->max_sweeps, opt->tol, opt->j_inner, C.d_sweeps + k,
                                C.d_eps + k, C.pgs);
      mark(kev, 4 * k + 2);
      launch_proximity<double>(st, nc, C.d_WH, C.d_pfree, C.d_f, h, C.d_p);  // Eq. 31
      mark(kev, 4 * k + 3);
      continue;
    }
    launch_directions(s, nc, k == 0);
    mark(kev, 4 * k);
    if (standard)
      build_WH_device(s, nc, C.d_nodes_c, C.d_W, false, C.d_C);   // W_k = J_k A^-1 J_k^T
    else if (mixed)
      launch_update_W<float>(st, nc, C.d_WH32, C.d_C, C.d_W32);
    else
      launch_update_W<double>(st, nc, C.d_WH, C.d_C, C.d_W);      // W_k = C_k W_H C_k^T
    mark(kev, 4 * k + 1);
    if (mixed)
      launch_pgs<float>(st, nc, C.d_W32, C.d_dk, C.d_mu, h, C.d_lam, C.d_status, opt->max_sweeps, opt->tol,
                        opt->j_inner, C.d_sweeps + k, C.d_eps + k, C.pgs);
    else
      launch_pgs<double>(st, nc, C.d_W, C.d_dk, C.d_mu, h, C.d_lam, C.d_status, opt->max_sweeps, opt->tol,
                         opt->j_inner, C.d_sweeps + k, C.d_eps + k, C.pgs);
    mark(kev, 4 * k + 2);
    if (standard) {
      launch_world_force(st, nc, C.d_C, C.d_lam, C.d_f);
      contact_force_solve(s, C.d_lam, S.d_sol);                      // A^-1 J_k^T lambda_k
      launch_standard_proximity(s, nc);                               // p_k = H (q_free + h^2 sol)
    } else if (mixed) {
      launch_world_force_proximity<float>(st, nc, C.d_C, C.d_lam, C.d_f, C.d_WH32, C.d_pfree, h, C.d_p);
    } else {
      launch_world_force_proximity<double>(st, nc, C.d_C, C.d_lam, C.d_f, C.d_WH, C.d_pfree, h, C.d_p);  // Eq. 31
    }
    mark(kev, 4 * k + 3);
  }
}

// The step after its Newton loop: corrective motion, integration (Eq. 20),
// the warm start of the next step.
void enqueue_post(icr_scene *s, const icr_step_opts *opt) {
  auto &C = s->con;
  auto &S = s->st;
  const int nc = opt->n_contacts;
  const bool standard = opt->scheme == 1;
  auto &Pr = s->pairs;
  const int P = Pr.count;
  auto mark = [&](int base, int i) {
    if (opt->timing) launch_stamp(s, base + i);
  };
  const int ev = kStampStep;
  mark(ev, 4);
  // corrective motion and integration (Eq. 20)
  if (P > 0) {
    launch_node_forces(s, nc, C.d_f, Pr.d_fu);                        // H_w^T f on the build's nodes
    contact_force_solve(s, Pr.d_fu, S.d_sol);
  } else if (!standard) {
    contact_force_solve(s, C.d_f, S.d_sol);                           // A^-1 H^T f (last W_H's Z)
  }
  launch_integrate(s);
  launch_store_forces(s, nc);   // and the time advance
  if (standard) launch_fill(s, C.d_WH, 9L * nc * nc, 0.0);           // no W_H in this scheme
  mark(ev, 5);
}

void enqueue_step(icr_scene *s, const icr_step_opts *opt) {
  enqueue_pre(s, opt);
  enqueue_newton(s, opt);
  enqueue_post(s, opt);
}

// icr_step's checks, buffers and per-step device parameters.
void step_prepare(icr_scene *s, const icr_obstacle *obs, const icr_step_opts *opt) {
  check_step(s, obs, opt);
  const int nc = opt->n_contacts;
  ensure_contact_buffers(s, nc);
  ensure_pair_step(s, nc);
  ensure_rhs_capacity(s, std::max(nc, s->pairs.count > 0 ? s->pairs.nu + nc - s->pairs.count : 0));
  if (opt->precision == ICR_FP32_IR) ensure_mixed(s);
  auto &S = s->st;
  if (!S.obs_valid || std::memcmp(&S.obs_host, obs, sizeof(icr_obstacle)) != 0) {
    launch_set_ctx(s, obs, nullptr);
    S.obs_host = *obs;
    S.obs_valid = true;
  }
}

// The host's record of an enqueued step.
void step_account(icr_scene *s, const icr_step_opts *opt) {
  auto &S = s->st;
  S.t = S.t + s->mesh.h;
  s->stepped = true;
  s->last_nc = opt->n_contacts;
  s->last_mixed = opt->precision == ICR_FP32_IR;
}

bool same_opts(const icr_step_opts &a, const icr_step_opts &b) {
  return a.n_contacts == b.n_contacts && a.n_newton == b.n_newton && a.max_sweeps == b.max_sweeps &&
         a.j_inner == b.j_inner && a.tol == b.tol && a.timing == b.timing && a.scheme == b.scheme &&
         a.precision == b.precision && a.refine == b.refine;
}

}  // namespace

icr_status icr_step(icr_scene *s, const icr_obstacle *obs, const icr_step_opts *opt, icr_step_report *rep) {
  return guarded(s, [&] {
    step_prepare(s, obs, opt);
    const int nc = opt->n_contacts;
    hipStream_t st = s->stream;
    auto &C = s->con;
    auto &S = s->st;
    const int nk = opt->n_newton;
    if (opt->graph) {
      auto &G = s->sg;
      if (!G.valid || G.epoch != s->epoch || !same_opts(G.key, *opt)) {
        G.reset();
        if (!G.cap) ICR_HIP(hipStreamCreateWithFlags(&G.cap, hipStreamNonBlocking));
        s->stream = G.cap;
        try {
          ICR_HIP(hipStreamBeginCapture(G.cap, hipStreamCaptureModeThreadLocal));
          enqueue_step(s, opt);
          ICR_HIP(hipStreamEndCapture(G.cap, &G.graph));
        } catch (...) {
          hipGraph_t junk = nullptr;
          (void)hipStreamEndCapture(G.cap, &junk);
          if (junk) (void)hipGraphDestroy(junk);
          s->stream = st;
          G.reset();
          throw;
        }
        s->stream = st;
        ICR_HIP(hipGraphInstantiate(&G.exec, G.graph, nullptr, nullptr, 0));
        G.key = *opt;
        G.epoch = s->epoch;
        G.valid = true;
      }
      ICR_HIP(hipGraphLaunch(G.exec, st));
    } else {
      enqueue_step(s, opt);
    }
    step_account(s, opt);
    if (rep) {
      std::memset(rep, 0, sizeof(*rep));
      rep->t = S.t;
      int nr = std::min(nk, 16);
      ICR_HIP(hipMemcpyAsync(rep->sweeps, C.d_sweeps, sizeof(int) * nr, hipMemcpyDeviceToHost, st));
      ICR_HIP(hipMemcpyAsync(rep->eps, C.d_eps, sizeof(double) * nr, hipMemcpyDeviceToHost, st));
      std::vector<int8_t> stat(nc);
      ICR_HIP(hipMemcpyAsync(stat.data(), C.d_status, nc, hipMemcpyDeviceToHost, st));
      ICR_HIP(hipStreamSynchronize(st));
      for (int8_t v : stat) {
        if (v == ICR_SEPARATE) rep->n_separate++;
        if (v == ICR_STICK) rep->n_stick++;
        if (v == ICR_SLIP) rep->n_slip++;
      }
      if (opt->timing) {
        std::vector<unsigned long long> ts(6 + 4 * nk);
        ICR_HIP(hipMemcpy(ts.data(), S.d_stamps, sizeof(unsigned long long) * ts.size(), hipMemcpyDeviceToHost));
        const double per_ms = s->clock_khz > 0 ? (double)s->clock_khz : 1e5;
        auto el = [&](int a, int b) { return (double)(long long)(ts[b] - ts[a]) / per_ms; };
        rep->ms_total = el(0, 5);
        rep->ms_free = el(0, 1);
        rep->ms_contacts = el(1, 2);
        rep->ms_build_WH = el(2, 3);
        rep->ms_newton = el(3, 4);
        rep->ms_correct = el(4, 5);
        for (int k = 0; k < nk; ++k) {
          rep->ms_update_W += el(6 + 4 * k, 6 + 4 * k + 1);
          rep->ms_pgs += el(6 + 4 * k + 1, 6 + 4 * k + 2);
          rep->ms_corr += el(6 + 4 * k + 2, 6 + 4 * k + 3);
        }
      }
    }
    return ICR_OK;
  });
}

icr_status icr_reserve(icr_scene *s, int32_t max_contacts, int32_t precision) {
  return guarded(s, [&] {
    if (!s->factored) throw StateError("icr_reserve before icr_factor");
    REQUIRE(max_contacts >= 1 && max_contacts <= kPgsMaxContacts, "max_contacts must be in [1, 4096]");
    REQUIRE(precision == ICR_FP64 || precision == ICR_FP32_IR, "precision must be ICR_FP64 or ICR_FP32_IR");
    ensure_contact_buffers(s, max_contacts);
    ensure_rhs_capacity(s, max_contacts);
    if (precision == ICR_FP32_IR) ensure_mixed(s);
    ICR_HIP(hipStreamSynchronize(s->stream));
    return ICR_OK;
  });
}

icr_status icr_get_state(icr_scene *s, double *q, double *v, double *t_out) {
  return guarded(s, [&] {
    if (!s->assembled) throw StateError("no mesh");
    const size_t bytes = sizeof(double) * s->mesh.n;
    if (q) ICR_HIP(hipMemcpyAsync(q, s->st.d_q, bytes, hipMemcpyDeviceToDevice, s->stream));
    if (v) ICR_HIP(hipMemcpyAsync(v, s->st.d_v, bytes, hipMemcpyDeviceToDevice, s->stream));
    if (t_out) *t_out = s->st.t;
    return ICR_OK;
  });
}

icr_status icr_set_state(icr_scene *s, const double *q, const double *v, double t) {
  return guarded(s, [&] {
    if (!s->assembled) throw StateError("no mesh");
    REQUIRE(q && v, "NULL device pointer");
    const size_t bytes = sizeof(double) * s->mesh.n;
    ICR_HIP(hipMemcpyAsync(s->st.d_q, q, bytes, hipMemcpyDeviceToDevice, s->stream));
    ICR_HIP(hipMemcpyAsync(s->st.d_v, v, bytes, hipMemcpyDeviceToDevice, s->stream));
    s->st.t = t;
    launch_set_ctx(s, nullptr, &t);
    launch_fill(s, s->st.d_node_force, (long)s->mesh.n, 0.0);   // a new trajectory: no warm start
    if (s->pairs.count > 0) launch_fill(s, s->pairs.d_force, 3L * s->pairs.count, 0.0);
    return ICR_OK;
  });
}

icr_status icr_get_step_results(icr_scene *s, int32_t *node_ids, double *q_free, double *p, double *lambda,
                                double *C, double *f, int8_t *status, double *WH) {
  return guarded(s, [&] {
    if (!s->stepped) throw StateError("no step has run");
    const int nc = s->last_nc;
    const size_t m = 3 * (size_t)nc;
    hipStream_t st = s->stream;
    auto cp = [&](void *dst, const void *src, size_t bytes) {
      if (dst) ICR_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st));
    };
    cp(node_ids, s->con.d_nodes_c, sizeof(int) * nc);
    cp(q_free, s->st.d_qfree, sizeof(double) * s->mesh.n);
    cp(p, s->con.d_p, sizeof(double) * m);
    cp(lambda, s->con.d_lam, sizeof(double) * m);
    cp(C, s->con.d_C, sizeof(double) * 9 * nc);
    cp(f, s->con.d_f, sizeof(double) * m);
    cp(status, s->con.d_status, nc);
    if (WH && s->last_mixed)
      launch_widen(s, s->con.d_WH32, WH, (long)(m * m));   // the step kept W_H in FP32
    else
      cp(WH, s->con.d_WH, sizeof(double) * m * m);
    return ICR_OK;
  });
}

icr_status icr_analyze(const double *nodes, int32_t N, const int32_t *tets, int32_t T, int32_t *perm, int32_t *sup,
                       int32_t nsup_cap, int32_t *rows_ptr, int32_t *rows, int32_t rows_cap, int32_t *nsup_out,
                       int32_t *nrows_out) {
  try {
    if (!nodes || !tets || N <= 0 || T <= 0) return ICR_E_ARG;
    for (long i = 0; i < 4L * T; ++i)
      if (tets[i] < 0 || tets[i] >= N) return ICR_E_ARG;
    MeshGraph g = build_graph(N, tets, T);
    Symbolic sym;
    analyze(nodes, g, 48, sym);
    if (!check_symbolic(g, sym).empty()) return ICR_E_HIP;
    if (nsup_out) *nsup_out = sym.nsup;
    if (nrows_out) *nrows_out = (int32_t)sym.rows.size();
    if (perm) std::copy(sym.perm.begin(), sym.perm.end(), perm);
    if (sup && rows_ptr && rows && sym.nsup <= nsup_cap && (int)sym.rows.size() <= rows_cap) {
      for (int s_ = 0; s_ < sym.nsup; ++s_) {
        sup[4 * s_] = sym.col0[s_];
        sup[4 * s_ + 1] = sym.ncol[s_];
        sup[4 * s_ + 2] = sym.parent[s_];
        sup[4 * s_ + 3] = sym.first_desc[s_];
      }
      std::copy(sym.rows_ptr.begin(), sym.rows_ptr.end(), rows_ptr);
      std::copy(sym.rows.begin(), sym.rows.end(), rows);
    }
    return ICR_OK;
  } catch (...) {
    return ICR_E_HIP;
  }
}

}  // extern "C"

namespace icr {

size_t newton_task_bytes() { return sizeof(NewtonTask); }

bool newton_batchable(const icr_scene *s, const icr_step_opts *opt) {
  return s && opt && opt->scheme == 0 && opt->precision == ICR_FP64 && !opt->timing && s->pairs.count == 0 &&
         opt->n_contacts >= 1 && opt->n_contacts <= kPgsWaveMax;
}

icr_status step_begin(icr_scene *s, const icr_obstacle *obs, const icr_step_opts *opt, void *task) {
  return guarded(s, [&] {
    if (!task) throw ArgError("step_begin: task is NULL");
    step_prepare(s, obs, opt);
    if (!newton_batchable(s, opt)) throw ArgError("step_begin: this step's Newton loop cannot run batched");
    enqueue_pre(s, opt);
    auto &C = s->con;
    NewtonTask t{};
    t.nc = opt->n_contacts;
    t.n_newton = opt->n_newton;
    t.max_sweeps = opt->max_sweeps;
    t.j_inner = opt->j_inner;
    t.tol = opt->tol;
    t.h = s->mesh.h;
    t.ctx = s->st.d_ctx;
    t.WH = C.d_WH;
    t.pfree = C.d_pfree;
    t.pstart = C.d_pstart;
    t.mu = C.d_mu;
    t.W = C.d_W;
    t.p = C.d_p;
    t.f = C.d_f;
    t.C = C.d_C;
    t.dk = C.d_dk;
    t.lam = C.d_lam;
    t.eps = C.d_eps;
    t.g = C.pgs.g;
    t.Wss = C.pgs.Wss;
    t.gnSet = C.pgs.gnSet;
    t.swn = C.pgs.swn;
    t.status = C.d_status;
    t.sweeps = C.d_sweeps;
    t.ctl = C.pgs.ctl;
    std::memcpy(task, &t, sizeof t);
    return ICR_OK;
  });
}

icr_status step_end(icr_scene *s, const icr_step_opts *opt) {
  return guarded(s, [&] {
    enqueue_post(s, opt);
    step_account(s, opt);
    return ICR_OK;
  });
}

icr_status newton_batch(void *stream, const void *tasks, const int *idx, int n, std::string &msg) {
  try {
    if (!tasks || !idx || n < 1 || n > kNewtonBatchMax) throw ArgError("newton_batch: 1..64 tasks");
    NewtonBatchIdx b{};
    b.n = n;
    for (int i = 0; i < n; ++i) b.idx[i] = idx[i];
    launch_newton_batch((hipStream_t)stream, static_cast<const NewtonTask *>(tasks), b);
    return ICR_OK;
  } catch (const ArgError &e) {
    msg = e.what();
    return ICR_E_ARG;
  } catch (const std::exception &e) {
    msg = e.what();
    return ICR_E_HIP;
  }
}

icr_status check_step_request(icr_scene *s, const icr_obstacle *obs, const icr_step_opts *opt, std::string &msg) {
  const icr_status st = guarded(s, [&] {
    check_step(s, obs, opt);
    return ICR_OK;
  });
  msg = s ? s->err : std::string("null scene");
  return st;
}

icr_status enqueue_eps_readback(icr_scene *s, int n_newton, double *dst) {
  return guarded(s, [&] {
    REQUIRE(n_newton >= 1 && n_newton <= kMaxNewton && s->con.d_eps, "no Newton iterations to read");
    ICR_HIP(hipMemcpyAsync(dst, s->con.d_eps, sizeof(double) * n_newton, hipMemcpyDeviceToHost, s->stream));
    return ICR_OK;
  });
}

int reserved_contacts(const icr_scene *s) { return s ? std::min(s->con.nc_cap, s->fac.nc_cap) : 0; }

int candidate_count(const icr_scene *s) { return (s && s->has_candidates) ? s->con.count : 0; }

void *scene_stream(const icr_scene *s) { return s ? (void *)s->stream : nullptr; }

bool mixed_reserved(const icr_scene *s) { return s && s->fac.have32 && s->fac.mixed_cap == s->fac.nc_cap; }

}  // namespace icr
