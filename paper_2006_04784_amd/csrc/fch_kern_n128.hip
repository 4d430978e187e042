// fch_kern_n128.hip -- compiled launch variants for N = 128 (row pass:
// rows per workgroup R, FFT elements per thread E, twiddles in LDS or not;
// column pass: E and twiddles in LDS or not).  The first of each list is the default.
#include "fch_variants.hpp"

FCH_VARIANTS(128, FCH_LIST(RowImpl<128, 2, 8, 1>::table(), RowImpl<128, 4, 8, 0>::table(), RowImpl<128, 2, 4, 0>::table()),
             FCH_LIST(ColImpl<128, 4, 0>::table(), ColImpl<128, 8, 0>::table(), ColImpl<128, 8, 1>::table()))
