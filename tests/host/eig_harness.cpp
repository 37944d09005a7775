// Runs the library's host eigen-decomposition (csrc/eig.h) on one matrix:
// reads n (int32) and the row-major n x n matrix from argv[1], writes ok
// (int32) and, when ok, lam (n), V (n x n) and V^{-1} (n x n) to argv[2].
#include <cstdio>
#include <string>
#include <vector>

#include "eig.h"

int main(int argc, char** argv) {
  if (argc != 3) return 2;
  FILE* f = fopen(argv[1], "rb");
  if (!f) return 2;
  int n = 0;
  if (fread(&n, 4, 1, f) != 1 || n < 1) return 2;
  std::vector<double> A((size_t)n * n), lam, V, Vi;
  if (fread(A.data(), 8, A.size(), f) != A.size()) return 2;
  fclose(f);
  std::string err;
  const int ok = grmhd::eig_real(n, A, &lam, &V, &Vi, &err) ? 1 : 0;
  FILE* o = fopen(argv[2], "wb");
  if (!o) return 2;
  fwrite(&ok, 4, 1, o);
  if (ok) {
    fwrite(lam.data(), 8, lam.size(), o);
    fwrite(V.data(), 8, V.size(), o);
    fwrite(Vi.data(), 8, Vi.size(), o);
  } else {
    fprintf(stderr, "%s\n", err.c_str());
  }
  fclose(o);
  return 0;
}
