// fch_kern_n16.hip -- compiled launch variants for N = 16 (row pass:
// rows per workgroup R, FFT elements per thread E, twiddles in LDS or not;
// column pass: E and twiddles in LDS or not).  The first of each list is the default.
#include "fch_variants.hpp"

FCH_VARIANTS(16, FCH_LIST(RowImpl<16, 2, 4, 1>::table(), RowImpl<16, 1, 4, 1>::table()),
             FCH_LIST(ColImpl<16, 4, 0>::table(), ColImpl<16, 4, 1>::table()))
