// Host analysis for the supernodal Cholesky of A = M + h B + h^2 K (Eq. 5):
// node graph of the tetrahedral mesh, nested-dissection ordering and the
// supernodal elimination structure that the dissection tree implies.
//
// Ordering: recursive coordinate bisection.  At each region the nodes are
// sorted along the axis of largest extent and cut near the median at the
// widest coordinate gap (between grid layers for the jittered grids); the
// vertex separator is the smaller of the two one-sided boundaries of the cut.
// Regions are numbered children first, separator last, so every supernode's
// subtree occupies a contiguous range of permuted nodes.
//
// Structure: the below-rows of a supernode are the nodes outside its region
// adjacent to it.  Because separators isolate sibling regions, these are all
// ancestor-separator nodes and contain the true fill of every column of the
// supernode; explicit zeros are stored and computed, which keeps the factor
// exact (relaxed supernodes = dissection tree nodes).
#include <algorithm>
#include <cmath>
#include <numeric>
#include <sstream>
#include <stdexcept>

#include "icr_internal.hpp"

namespace icr {

MeshGraph build_graph(int N, const int32_t *tets, int T) {
  MeshGraph g;
  g.N = N;
  std::vector<std::vector<int>> nb(N);
  for (int i = 0; i < N; ++i) nb[i].push_back(i);
  for (int t = 0; t < T; ++t)
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b)
        if (a != b) nb[tets[4 * t + a]].push_back(tets[4 * t + b]);
  g.ptr.assign(N + 1, 0);
  for (int i = 0; i < N; ++i) {
    auto &v = nb[i];
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
    g.ptr[i + 1] = g.ptr[i] + (int)v.size();
  }
  g.adj.resize(g.ptr[N]);
  for (int i = 0; i < N; ++i) std::copy(nb[i].begin(), nb[i].end(), g.adj.begin() + g.ptr[i]);
  return g;
}

namespace {

struct ND {
  const double *xyz;
  const MeshGraph *g;
  int leaf_max;
  std::vector<int> stamp;   // region marker
  int cur = 0;
  Symbolic *sym;
  int next_pos = 0;
  std::vector<std::vector<int>> kids;

  int make_sup(const std::vector<int> &nodes, const std::vector<int> &children) {
    int s = sym->nsup++;
    sym->col0.push_back(next_pos);
    sym->ncol.push_back((int)nodes.size());
    sym->parent.push_back(-1);
    sym->first_desc.push_back(children.empty() ? s : sym->first_desc[children[0]]);
    for (int c : children) sym->parent[c] = s;
    kids.push_back(children);
    for (int v : nodes) sym->perm[next_pos++] = v;
    return s;
  }

  int rec(std::vector<int> nodes) {
    const int n = (int)nodes.size();
    if (n <= leaf_max) {
      std::sort(nodes.begin(), nodes.end());
      return make_sup(nodes, {});
    }
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int v : nodes)
      for (int a = 0; a < 3; ++a) {
        lo[a] = std::min(lo[a], xyz[3 * v + a]);
        hi[a] = std::max(hi[a], xyz[3 * v + a]);
      }
    int ax = 0;
    for (int a = 1; a < 3; ++a)
      if (hi[a] - lo[a] > hi[ax] - lo[ax]) ax = a;
    std::stable_sort(nodes.begin(), nodes.end(), [&](int u, int v) {
      double cu = xyz[3 * u + ax], cv = xyz[3 * v + ax];
      return cu < cv || (cu == cv && u < v);
    });
    int k0 = std::max(1, (int)(0.35 * n)), k1 = std::min(n - 1, (int)(0.65 * n));
    int best = n / 2;
    double bgap = -1.0;
    for (int k = k0; k <= k1; ++k) {
      double gap = xyz[3 * nodes[k] + ax] - xyz[3 * nodes[k - 1] + ax];
      if (gap > bgap * (1.0 + 1e-9) ||
          (std::fabs(gap - bgap) <= 1e-9 * std::fabs(bgap) && std::abs(k - n / 2) < std::abs(best - n / 2))) {
        bgap = gap;
        best = k;
      }
    }
    // mark right side
    ++cur;
    const int right = cur;
    for (int k = best; k < n; ++k) stamp[nodes[k]] = right;
    std::vector<int> sepL, sepR;
    ++cur;
    const int left = cur;
    for (int k = 0; k < best; ++k) stamp[nodes[k]] = left;
    for (int k = 0; k < best; ++k) {
      int v = nodes[k];
      for (int e = g->ptr[v]; e < g->ptr[v + 1]; ++e)
        if (stamp[g->adj[e]] == right) {
          sepL.push_back(v);
          break;
        }
    }
    for (int k = best; k < n; ++k) {
      int v = nodes[k];
      for (int e = g->ptr[v]; e < g->ptr[v + 1]; ++e)
        if (stamp[g->adj[e]] == left) {
          sepR.push_back(v);
          break;
        }
    }
    std::vector<int> A, B, S;
    bool useL = sepL.size() <= sepR.size();
    ++cur;
    const int sepmark = cur;
    for (int v : (useL ? sepL : sepR)) stamp[v] = sepmark;
    for (int k = 0; k < n; ++k) {
      int v = nodes[k];
      if (stamp[v] == sepmark)
        S.push_back(v);
      else if (k < best)
        A.push_back(v);
      else
        B.push_back(v);
    }
    if (S.empty()) {  // disconnected halves: any single node separates them
      if (!A.empty()) {
        S.push_back(A.back());
        A.pop_back();
      } else {
        S.push_back(B.back());
        B.pop_back();
      }
    }
    std::sort(S.begin(), S.end());
    std::vector<int> children;
    if (!A.empty()) children.push_back(rec(std::move(A)));
    if (!B.empty()) children.push_back(rec(std::move(B)));
    return make_sup(S, children);
  }
};

}  // namespace

void analyze(const double *xyz, const MeshGraph &g, int leaf_max, Symbolic &sym) {
  const int N = g.N;
  sym = Symbolic();
  sym.N = N;
  sym.perm.assign(N, -1);
  ND nd;
  nd.xyz = xyz;
  nd.g = &g;
  nd.leaf_max = leaf_max;
  nd.stamp.assign(N, 0);
  nd.sym = &sym;
  // connected components are dissected separately and become sibling roots
  std::vector<int> comp(N, -1);
  std::vector<std::vector<int>> comps;
  for (int s = 0; s < N; ++s) {
    if (comp[s] >= 0) continue;
    std::vector<int> stack{s}, members;
    comp[s] = (int)comps.size();
    while (!stack.empty()) {
      int v = stack.back();
      stack.pop_back();
      members.push_back(v);
      for (int e = g.ptr[v]; e < g.ptr[v + 1]; ++e) {
        int u = g.adj[e];
        if (comp[u] < 0) {
          comp[u] = comp[s];
          stack.push_back(u);
        }
      }
    }
    comps.push_back(std::move(members));
  }
  for (auto &c : comps) nd.rec(c);
  sym.iperm.assign(N, -1);
  for (int p = 0; p < N; ++p) sym.iperm[sym.perm[p]] = p;

  const int ns = sym.nsup;
  sym.child_ptr.assign(ns + 1, 0);
  for (int s = 0; s < ns; ++s) sym.child_ptr[s + 1] = sym.child_ptr[s] + (int)nd.kids[s].size();
  sym.child.clear();
  for (int s = 0; s < ns; ++s)
    for (int c : nd.kids[s]) sym.child.push_back(c);

  // below rows: nodes outside the region adjacent to it (all later in the order)
  sym.rows_ptr.assign(ns + 1, 0);
  sym.rows.clear();
  std::vector<int> mark(N, -1);
  for (int s = 0; s < ns; ++s) {
    int rlo = sym.col0[sym.first_desc[s]], rhi = sym.col0[s] + sym.ncol[s];
    std::vector<int> r;
    for (int p = rlo; p < rhi; ++p) {
      int v = sym.perm[p];
      for (int e = g.ptr[v]; e < g.ptr[v + 1]; ++e) {
        int q = sym.iperm[g.adj[e]];
        if (q >= rhi && mark[q] != s) {
          mark[q] = s;
          r.push_back(q);
        }
        if (q < rlo) throw std::runtime_error("dissection: region adjacent to an earlier node");
      }
    }
    std::sort(r.begin(), r.end());
    sym.rows.insert(sym.rows.end(), r.begin(), r.end());
    sym.rows_ptr[s + 1] = (int)sym.rows.size();
  }
  // heights and levels
  sym.height.assign(ns, 0);
  int H = 0;
  for (int s = 0; s < ns; ++s) {
    int h = 0;
    for (int e = sym.child_ptr[s]; e < sym.child_ptr[s + 1]; ++e) h = std::max(h, sym.height[sym.child[e]] + 1);
    sym.height[s] = h;
    H = std::max(H, h);
  }
  sym.nlevels = H + 1;
  sym.level_ptr.assign(H + 2, 0);
  for (int s = 0; s < ns; ++s) sym.level_ptr[sym.height[s] + 1]++;
  for (int l = 0; l <= H; ++l) sym.level_ptr[l + 1] += sym.level_ptr[l];
  sym.level_sup.assign(ns, 0);
  std::vector<int> fill(sym.level_ptr.begin(), sym.level_ptr.end() - 1);
  for (int s = 0; s < ns; ++s) sym.level_sup[fill[sym.height[s]]++] = s;
}

std::string check_symbolic(const MeshGraph &g, const Symbolic &sym) {
  std::ostringstream err;
  const int N = sym.N;
  std::vector<int> seen(N, 0);
  for (int p = 0; p < N; ++p) {
    int v = sym.perm[p];
    if (v < 0 || v >= N || seen[v]++) {
      err << "perm is not a permutation at " << p;
      return err.str();
    }
  }
  int pos = 0;
  for (int s = 0; s < sym.nsup; ++s) {
    if (sym.col0[s] != pos || sym.ncol[s] < 1) {
      err << "supernode " << s << " columns not contiguous";
      return err.str();
    }
    pos += sym.ncol[s];
    int p = sym.parent[s];
    if (p >= 0 && p <= s) {
      err << "parent not after child at " << s;
      return err.str();
    }
    if (p >= 0) {
      // child's below rows must be columns or below rows of the parent
      int pc0 = sym.col0[p], pc1 = pc0 + sym.ncol[p];
      for (int e = sym.rows_ptr[s]; e < sym.rows_ptr[s + 1]; ++e) {
        int r = sym.rows[e];
        bool ok = (r >= pc0 && r < pc1) ||
                  std::binary_search(sym.rows.begin() + sym.rows_ptr[p], sym.rows.begin() + sym.rows_ptr[p + 1], r);
        if (!ok) {
          err << "row " << r << " of supernode " << s << " missing in parent " << p;
          return err.str();
        }
      }
    } else if (sym.rows_ptr[s + 1] != sym.rows_ptr[s]) {
      err << "root " << s << " has below rows";
      return err.str();
    }
  }
  if (pos != N) return "columns do not cover all nodes";
  (void)g;
  return std::string();
}

}  // namespace icr
