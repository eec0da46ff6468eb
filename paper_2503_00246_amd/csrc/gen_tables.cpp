// Build-time generator of the 1D tables as compile-time constants for the box kernel:
//   gen_tables OUT.h
// writes, for every degree k = 1..kMaxDegree, the reference jump vectors (k x (2k+1), row j-1 = order
// j), the reference mass matrix ((k+1) x (k+1)), the reference stiffness matrix (the interior-cell
// Laplacian's 1D factor) and the order coupling H of the macro-patch form (k x k), computed by
// tables_1d / stiffness_1d / macro_mix_1d in long double and rounded
// once to double, as hexadecimal floating literals (exact).  The kernels fold them into immediates,
// so the face pipeline reads no table from memory.
#include <cstdio>
#include <vector>

#include "ghost_config.h"
#include "ghost_plan.h"

int main(int argc, char **argv) {
  if (argc != 2) {
    std::fprintf(stderr, "usage: %s OUT.h\n", argv[0]);
    return 2;
  }
  std::FILE *f = std::fopen(argv[1], "w");
  if (!f) return 1;
  std::fprintf(f, "// Generated at build time by gen_tables.cpp from tables_1d; not edited by hand.\n");
  std::fprintf(f, "#pragma once\n\nnamespace ghost {\nnamespace gen {\n\ntemplate <int K>\nstruct Tab1d;\n\n");
  for (int k = 1; k <= ghost::kMaxDegree; ++k) {
    std::vector<long double> nodes, weights, jumps, mass;
    ghost::tables_1d(k, nodes, weights, jumps, mass);
    std::fprintf(f, "template <>\nstruct Tab1d<%d> {\n  static constexpr double g[%zu] = {", k + 1, jumps.size());
    for (size_t i = 0; i < jumps.size(); ++i) std::fprintf(f, "%s%a", i ? ", " : "", (double)jumps[i]);
    std::fprintf(f, "};\n  static constexpr double M[%zu] = {", mass.size());
    for (size_t i = 0; i < mass.size(); ++i) std::fprintf(f, "%s%a", i ? ", " : "", (double)mass[i]);
    std::vector<long double> stiff;
    ghost::stiffness_1d(k, stiff);
    std::fprintf(f, "};\n  static constexpr double A[%zu] = {", stiff.size());
    for (size_t i = 0; i < stiff.size(); ++i) std::fprintf(f, "%s%a", i ? ", " : "", (double)stiff[i]);
    std::vector<long double> mix;
    ghost::macro_mix_1d(k, mix);
    std::fprintf(f, "};\n  static constexpr double H[%zu] = {", mix.size());
    for (size_t i = 0; i < mix.size(); ++i) std::fprintf(f, "%s%a", i ? ", " : "", (double)mix[i]);
    std::fprintf(f, "};\n};\n\n");
  }
  std::fprintf(f, "}  // namespace gen\n}  // namespace ghost\n");
  return std::fclose(f) == 0 ? 0 : 1;
}
