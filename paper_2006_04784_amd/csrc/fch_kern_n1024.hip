// fch_kern_n1024.hip -- compiled launch variants for N = 1024 (row pass:
// rows per workgroup R, FFT elements per thread E, twiddles in LDS or not;
// column pass: E and twiddles in LDS or not).  The first of each list is the default.
#include "fch_variants.hpp"

FCH_VARIANTS(1024, FCH_LIST(RowImpl<1024, 2, 8, 0>::table(), RowImpl<1024, 4, 16, 1>::table(), RowImpl<1024, 4, 16, 0>::table(), RowImpl<1024, 2, 16, 0>::table(), RowImpl<1024, 4, 8, 0>::table(), RowImpl<1024, 1, 8, 0>::table(), RowImpl<1024, 2, 4, 0>::table(), RowImpl<1024, 8, 16, 0>::table()),
             FCH_LIST(ColImpl<1024, 4, 0>::table(), ColImpl<1024, 4, 1>::table(), ColImpl<1024, 8, 0>::table()))
FCH_PSD_SOLVE(1024, 2, 8, 0, 4, 0, 2)
