// Host-only driver of the library's mesh analysis (nested dissection and
// supernodal symbolic structure), built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_host_library.py.
//
// Input file (little-endian): int32 N, int32 T, N*3 float64 node positions,
// T*4 int32 tetrahedra.  Prints "ok <supernodes> <below rows>" when the
// structure passes the library's own consistency check, else the message.
#include <cstdio>
#include <vector>

#include "icr_internal.hpp"

int main(int argc, char **argv) {
  if (argc != 2) {
    std::fprintf(stderr, "usage: %s mesh.bin\n", argv[0]);
    return 2;
  }
  std::FILE *f = std::fopen(argv[1], "rb");
  if (!f) return 2;
  int32_t N = 0, T = 0;
  if (std::fread(&N, 4, 1, f) != 1 || std::fread(&T, 4, 1, f) != 1 || N <= 0 || T <= 0) return 2;
  std::vector<double> xyz(3 * (size_t)N);
  std::vector<int32_t> tets(4 * (size_t)T);
  if (std::fread(xyz.data(), 8, xyz.size(), f) != xyz.size()) return 2;
  if (std::fread(tets.data(), 4, tets.size(), f) != tets.size()) return 2;
  std::fclose(f);
  icr::MeshGraph g = icr::build_graph(N, tets.data(), T);
  icr::Symbolic sym;
  icr::analyze(xyz.data(), g, 48, sym);
  const std::string bad = icr::check_symbolic(g, sym);
  if (!bad.empty()) {
    std::printf("%s\n", bad.c_str());
    return 1;
  }
  std::printf("ok %d %zu\n", sym.nsup, sym.rows.size());
  return 0;
}
