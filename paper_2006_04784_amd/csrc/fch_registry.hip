// fch_registry.hip -- the compiled launch variants per grid size.
#include "fch_kernels.hpp"

namespace fch {

#define FCH_DECL(N)                                \
  const RowVT* const* row_variants_##N(int* n);    \
  const ColVT* const* col_variants_##N(int* n);    \
  const PsdSolveVT* psd_solve_##N();
FCH_DECL(16)
FCH_DECL(32)
FCH_DECL(64)
FCH_DECL(128)
FCH_DECL(256)
FCH_DECL(512)
FCH_DECL(1024)
FCH_DECL(2048)
FCH_DECL(4096)
#undef FCH_DECL

static const RowVT* const* rows_for(int N, int* n) {
  switch (N) {
    case 16: return row_variants_16(n);
    case 32: return row_variants_32(n);
    case 64: return row_variants_64(n);
    case 128: return row_variants_128(n);
    case 256: return row_variants_256(n);
    case 512: return row_variants_512(n);
    case 1024: return row_variants_1024(n);
    case 2048: return row_variants_2048(n);
    case 4096: return row_variants_4096(n);
  }
  *n = 0;
  return nullptr;
}
static const ColVT* const* cols_for(int N, int* n) {
  switch (N) {
    case 16: return col_variants_16(n);
    case 32: return col_variants_32(n);
    case 64: return col_variants_64(n);
    case 128: return col_variants_128(n);
    case 256: return col_variants_256(n);
    case 512: return col_variants_512(n);
    case 1024: return col_variants_1024(n);
    case 2048: return col_variants_2048(n);
    case 4096: return col_variants_4096(n);
  }
  *n = 0;
  return nullptr;
}

const PsdSolveVT* psd_solve_variant(int N) {
  switch (N) {
    case 256: return psd_solve_256();
    case 512: return psd_solve_512();
    case 1024: return psd_solve_1024();
    case 2048: return psd_solve_2048();
  }
  return nullptr;
}

int row_variant_count(int N) {
  int n = 0;
  rows_for(N, &n);
  return n;
}
const RowVT* row_variant(int N, int i) {
  int n = 0;
  const RowVT* const* v = rows_for(N, &n);
  return (v && i >= 0 && i < n) ? v[i] : nullptr;
}
int col_variant_count(int N) {
  int n = 0;
  cols_for(N, &n);
  return n;
}
const ColVT* col_variant(int N, int i) {
  int n = 0;
  const ColVT* const* v = cols_for(N, &n);
  return (v && i >= 0 && i < n) ? v[i] : nullptr;
}

}  // namespace fch
