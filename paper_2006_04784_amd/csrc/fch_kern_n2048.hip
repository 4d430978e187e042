// fch_kern_n2048.hip -- compiled launch variants for N = 2048 (row pass:
// rows per workgroup R, FFT elements per thread E, twiddles in LDS or not;
// column pass: E and twiddles in LDS or not).  The first of each list is the default.
#include "fch_variants.hpp"

FCH_VARIANTS(2048, FCH_LIST(RowImpl<2048, 2, 16, 0>::table(), RowImpl<2048, 2, 16, 1>::table(), RowImpl<2048, 2, 8, 0>::table(), RowImpl<2048, 1, 16, 0>::table(), RowImpl<2048, 1, 8, 0>::table()),
             FCH_LIST(ColImpl<2048, 8, 0>::table(), ColImpl<2048, 4, 0>::table(), ColImpl<2048, 8, 1>::table()))
FCH_PSD_SOLVE(2048, 2, 16, 0, 8, 0, 1)
