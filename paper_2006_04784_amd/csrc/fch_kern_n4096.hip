// fch_kern_n4096.hip -- compiled launch variants for N = 4096 (row pass:
// rows per workgroup R, FFT elements per thread E, twiddles in LDS or not;
// column pass: E and twiddles in LDS or not).  The first of each list is the default.
// One column (two sequences of 4096 points) fills 147 KB of LDS; the fused
// column epilogues spill registers at this size (correct, not tuned).
#include "fch_variants.hpp"

FCH_VARIANTS(4096, FCH_LIST(RowImpl<4096, 1, 16, 0>::table(), RowImpl<4096, 1, 8, 0>::table()),
             FCH_LIST(ColImpl<4096, 8, 0>::table()))
