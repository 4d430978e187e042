// fch_kern_n64.hip -- compiled launch variants for N = 64 (row pass:
// rows per workgroup R, FFT elements per thread E, twiddles in LDS or not;
// column pass: E and twiddles in LDS or not).  The first of each list is the default.
#include "fch_variants.hpp"

FCH_VARIANTS(64, FCH_LIST(RowImpl<64, 2, 8, 1>::table(), RowImpl<64, 4, 8, 0>::table(), RowImpl<64, 2, 4, 0>::table()),
             FCH_LIST(ColImpl<64, 4, 0>::table(), ColImpl<64, 8, 0>::table(), ColImpl<64, 8, 1>::table()))
