// fch_kern_n32.hip -- compiled launch variants for N = 32 (row pass:
// rows per workgroup R, FFT elements per thread E, twiddles in LDS or not;
// column pass: E and twiddles in LDS or not).  The first of each list is the default.
#include "fch_variants.hpp"

FCH_VARIANTS(32, FCH_LIST(RowImpl<32, 2, 4, 1>::table(), RowImpl<32, 4, 4, 1>::table()),
             FCH_LIST(ColImpl<32, 4, 0>::table(), ColImpl<32, 4, 1>::table()))
