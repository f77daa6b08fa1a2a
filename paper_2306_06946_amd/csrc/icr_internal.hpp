// Internal declarations shared by the library's host planning code and HIP
// kernels.  Nothing here is part of the public ABI (include/icr.h).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "icr.h"

namespace icr {

// ---------------------------------------------------------------------------
// Host analysis: mesh graph, nested dissection, supernodal symbolic structure
// ---------------------------------------------------------------------------

struct MeshGraph {
  int N = 0;
  std::vector<int> ptr;  // N+1
  std::vector<int> adj;  // sorted neighbours, self included
};

// Per supernode, in postorder (children before parents).  Columns of a
// supernode are the consecutive permuted nodes [col0, col0 + ncol); its region
// (all nodes of its subtree) is [col0[first_desc], col0 + ncol).
struct Symbolic {
  int N = 0;
  std::vector<int> perm, iperm;             // perm[new] = old, iperm[old] = new
  int nsup = 0;
  std::vector<int> col0, ncol, parent, first_desc, height;
  std::vector<int> rows_ptr, rows;          // below-row permuted nodes (sorted, > cols)
  std::vector<int> child_ptr, child;        // children of each supernode, ascending
  std::vector<int> level_ptr, level_sup;    // supernodes grouped by height
  int nlevels = 0;
};

MeshGraph build_graph(int N, const int32_t *tets, int T);
// Nested dissection on node coordinates + graph separators, then the
// supernodal structure implied by the dissection tree.
void analyze(const double *xyz, const MeshGraph &g, int leaf_max, Symbolic &sym);
// Consistency checks (permutation, containment of child structure in parent);
// returns an empty string when valid.
std::string check_symbolic(const MeshGraph &g, const Symbolic &sym);

// ---------------------------------------------------------------------------
// Device-side descriptors
// ---------------------------------------------------------------------------

// One supernode as seen by the kernels.  DOF-level: n_s = 3*ncol columns,
// f_s = 3*(ncol + nb) front rows.
struct SupDev {
  int col0;       // first permuted node
  int ncol;       // nodes in the supernode
  int nb;         // below-row nodes
  int parent;     // -1 for a root
  int rows_off;   // into rows[] (below-row permuted nodes)
  int first_desc; // postorder index of the first descendant
  int child_off;  // into child[] / invmap_off[]
  int nchild;
  int region_nodes;   // nodes in the subtree region
  int pad;
  long long front_off;   // doubles, F_s (f_s x f_s, column-major)
  long long linv_off;    // doubles, L_ss^{-1} (n_s x n_s, column-major)
  long long x_off;       // doubles, multi-RHS front X_s (f_s x rmax_s)
  long long z_off;       // doubles, Z_s (n_s x rmax_s)
  long long x1_off;      // doubles, single-RHS front (f_s)
  int rmax;              // RHS column capacity of X_s / Z_s
  int pad2;
};

// Entry of the A -> front scatter list: front of supernode `s`, local node
// row `lr` (in cols then below rows), local node column `lc`, BSR block `blk`.
struct AScatter {
  int s, lr, lc, blk;
};

}  // namespace icr
