// Host code of the library under AddressSanitizer and UBSan (built by
// tests/test_host_sanitizers.py with g++, no GPU): every Trefftz table
// (n = 1..3, p = 1..10, the three seed bases), then, for each mesh file given
// on the command line, the topology, the tent pitcher and the simplex rules.
// Mesh file: int32 dim, nv, ne; float64 T, gamma; coords (nv x dim, float64),
// elements (ne x (dim + 1), int32), speeds (ne, float64).
#include <cstdio>
#include <vector>

#include "trefftz_table.h"

int main(int argc, char** argv) {
  long long entries = 0;
  for (int n = 1; n <= 3; ++n)
    for (int seed = 0; seed <= 2; ++seed)
      for (int p = 1; p <= 10; ++p) {
        const tdg::Table T = tdg::build_table(n, p, seed);
        entries += (long long)(T.fo_idx.size() + T.u_idx.size() + T.ue_idx.size() + T.tr_j.size());
      }
  std::printf("tables %lld\n", entries);
  for (int a = 1; a < argc; ++a) {
    FILE* f = std::fopen(argv[a], "rb");
    if (!f) return 3;
    int32_t dim = 0, nv = 0, ne = 0;
    double T = 0, gamma = 0;
    bool ok = std::fread(&dim, 4, 1, f) == 1 && std::fread(&nv, 4, 1, f) == 1 && std::fread(&ne, 4, 1, f) == 1 &&
              std::fread(&T, 8, 1, f) == 1 && std::fread(&gamma, 8, 1, f) == 1;
    std::vector<double> X(ok ? (size_t)nv * dim : 0), c(ok ? (size_t)ne : 0);
    std::vector<int32_t> E(ok ? (size_t)ne * (dim + 1) : 0);
    ok = ok && std::fread(X.data(), 8, X.size(), f) == X.size() && std::fread(E.data(), 4, E.size(), f) == E.size() &&
         std::fread(c.data(), 8, c.size(), f) == c.size();
    std::fclose(f);
    if (!ok) return 3;
    tdg_mesh m{};
    m.dim = dim;
    m.nv = nv;
    m.ne = ne;
    m.coords = X.data();
    m.elems = E.data();
    m.bface_kind = nullptr;
    tdg::Topology topo;
    std::string err;
    if (tdg::build_topology(m, c.data(), topo, err)) return 4;
    tdg::TentList tl;
    if (tdg::pitch_tents(topo, T, gamma, tl, err)) return 5;
    for (int q = 1; q <= 10; ++q) tdg::simplex_rule(dim, q);
    std::printf("mesh %d %zu %zu\n", a, tl.V.size(), tl.layer_ptr.size() - 1);
  }
  return 0;
}
