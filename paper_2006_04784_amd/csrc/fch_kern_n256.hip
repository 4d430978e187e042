// fch_kern_n256.hip -- compiled launch variants for N = 256 (row pass:
// rows per workgroup R, FFT elements per thread E, twiddles in LDS or not;
// column pass: E and twiddles in LDS or not).  The first of each list is the default.
#include "fch_variants.hpp"

FCH_VARIANTS(256, FCH_LIST(RowImpl<256, 2, 8, 0>::table(), RowImpl<256, 2, 16, 1>::table(), RowImpl<256, 4, 8, 0>::table(), RowImpl<256, 4, 16, 0>::table(), RowImpl<256, 1, 8, 0>::table(), RowImpl<256, 8, 4, 0>::table()),
             FCH_LIST(ColImpl<256, 4, 0>::table(), ColImpl<256, 4, 1>::table(), ColImpl<256, 8, 0>::table()))
FCH_PSD_SOLVE(256, 2, 8, 0, 4, 0, 2)
