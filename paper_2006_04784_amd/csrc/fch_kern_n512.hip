// fch_kern_n512.hip -- compiled launch variants for N = 512 (row pass:
// rows per workgroup R, FFT elements per thread E, twiddles in LDS or not;
// column pass: E and twiddles in LDS or not).  The first of each list is the default.
#include "fch_variants.hpp"

FCH_VARIANTS(512, FCH_LIST(RowImpl<512, 2, 8, 0>::table(), RowImpl<512, 2, 8, 1>::table(), RowImpl<512, 4, 8, 0>::table(), RowImpl<512, 2, 16, 0>::table(), RowImpl<512, 2, 4, 0>::table(), RowImpl<512, 8, 8, 0>::table()),
             FCH_LIST(ColImpl<512, 4, 0>::table(), ColImpl<512, 4, 1>::table(), ColImpl<512, 8, 0>::table()))
FCH_PSD_SOLVE(512, 2, 8, 0, 4, 0, 2)
