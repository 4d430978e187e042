// fch_variants.hpp -- launch wrappers of the kernel templates for one grid
// size; each fch_kern_n<N>.hip instantiates the variants of its N.
#pragma once
#include <hip/hip_ext.h>

#include "fch_kernels_impl.hpp"

// launch, optionally with start and/or stop events attached to the dispatch
// itself (either may be null)
#define FCH_LAUNCH(K, GRID, BLOCK, S, E0, E1, ...)                                   \
  do {                                                                                \
    if ((E0) || (E1))                                                                 \
      hipExtLaunchKernelGGL(K, GRID, BLOCK, 0, S, E0, E1, 0, __VA_ARGS__);            \
    else                                                                              \
      hipLaunchKernelGGL(K, GRID, BLOCK, 0, S, __VA_ARGS__);                          \
  } while (0)

namespace fch {

template <int N, int R, int E, int TWL>
struct RowImpl {
  static constexpr int NT = R * (N / E);
  static hipError_t row(int mode, const RowArgs& a, hipStream_t s, hipEvent_t e0,
                        hipEvent_t e1) {
    const int* done = (mode == ROW_MU && a.check_done) ? &a.ctl->done : nullptr;
    const int* nodone = nullptr;
    switch (mode) {
      case ROW_MU:
        FCH_LAUNCH((k_row<N, R, E, ROW_MU, TWL>), dim3(N / R), dim3(NT), s, e0, e1, a, done);
        break;
      case ROW_FWD:
        FCH_LAUNCH((k_row<N, R, E, ROW_FWD, TWL>), dim3(N / (2 * R)), dim3(NT), s, e0, e1, a,
                   nodone);
        break;
      case ROW_INV:
        FCH_LAUNCH((k_row<N, R, E, ROW_INV, TWL>), dim3(N / (2 * R)), dim3(NT), s, e0, e1, a,
                   nodone);
        break;
      default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  static hipError_t row_ens(EnsMember* m, int first, int count, int mode, hipStream_t s) {
    switch (mode) {
      case ENS_ROW:
        hipLaunchKernelGGL((k_row_ens<N, R, E, TWL, ENS_ROW>), dim3(N / R, count), dim3(NT), 0, s,
                           m, first);
        break;
      case ENS_ROW_TRACK:
        hipLaunchKernelGGL((k_row_ens<N, R, E, TWL, ENS_ROW_TRACK>), dim3(N / R, count), dim3(NT),
                           0, s, m, first);
        break;
      case ENS_ROW_PSD:
        hipLaunchKernelGGL((k_row_ens<N, R, E, TWL, ENS_ROW_PSD>), dim3(N / R, count), dim3(NT), 0,
                           s, m, first);
        break;
      default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  static hipError_t row_batch(int mode, const RowArgs& a, int batch, size_t pstride,
                              size_t sstride, hipStream_t s) {
    const dim3 grid(N / (2 * R), batch);
    if (mode == ROW_FWD)
      hipLaunchKernelGGL((k_row_b<N, R, E, ROW_FWD, TWL>), grid, dim3(NT), 0, s, a, pstride,
                         sstride);
    else if (mode == ROW_INV)
      hipLaunchKernelGGL((k_row_b<N, R, E, ROW_INV, TWL>), grid, dim3(NT), 0, s, a, pstride,
                         sstride);
    else
      return hipErrorInvalidValue;
    return hipGetLastError();
  }
  static const RowVT* table() {
    static const RowVT vt = {N, R, E, TWL, NT, &row, &row_ens, &row_batch};
    return &vt;
  }
};

template <int N, int E, int TWL>
struct ColImpl {
  static constexpr int CT = N / E;
  static constexpr int H = N / 2 + 1;
  // At N = 4096 the fused passes (those with an epilogue) run as two
  // launches, the columns kx >= 1 and the self-conjugate pair, so that neither
  // path holds the other's registers: compiled as one kernel, the pair's path
  // (both of its columns' state values) sets the register count of every
  // workgroup and spilled up to 1.1 KB per lane to scratch.  The pair's single
  // workgroup runs on the plan's side stream beside the others.  (At 2048 the
  // split measured slower: the others fill every CU first, and the pair's
  // workgroup, started late, outlasts them.  Holding both launches to two
  // waves per SIMD, so that the pair shares a CU, made the pair spill and
  // was slower still.)
  template <int EPI>
  static constexpr bool SPLIT = (N >= 4096 && EPI != EPI_NONE);
  static constexpr int EP = E;  // elements per thread of the pair's launch

  template <int EPI, int PRO>
  static hipError_t lc(const ColArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
                       const SideLane* side) {
    const int* done = a.check_done ? &a.ctl->done : nullptr;
    if constexpr (SPLIT<EPI>) {
      hipError_t err;
      if (side && side->stream) {
        if ((err = hipEventRecord(side->fork, s)) != hipSuccess) return err;
        if ((err = hipStreamWaitEvent(side->stream, side->fork, 0)) != hipSuccess) return err;
        hipLaunchKernelGGL((k_col<N, EP, EPI, PRO, TWL, 2>), dim3(1), dim3(N / EP), 0,
                           side->stream, a, done);
        if ((err = hipGetLastError()) != hipSuccess) return err;
        if ((err = hipEventRecord(side->join, side->stream)) != hipSuccess) return err;
        FCH_LAUNCH((k_col<N, E, EPI, PRO, TWL, 1>), dim3(N / 2 - 1), dim3(CT), s, e0, e1, a,
                   done);
        if ((err = hipGetLastError()) != hipSuccess) return err;
        return hipStreamWaitEvent(s, side->join, 0);
      }
      FCH_LAUNCH((k_col<N, E, EPI, PRO, TWL, 1>), dim3(N / 2 - 1), dim3(CT), s, e0, nullptr, a,
                 done);
      FCH_LAUNCH((k_col<N, EP, EPI, PRO, TWL, 2>), dim3(1), dim3(N / EP), s, nullptr, e1, a,
                 done);
    } else {
      FCH_LAUNCH((k_col<N, E, EPI, PRO, TWL>), dim3(N / 2), dim3(CT), s, e0, e1, a, done);
    }
    return hipGetLastError();
  }

  static hipError_t col(int epi, int pro, const ColArgs& a, hipStream_t s, hipEvent_t e0,
                        hipEvent_t e1, const SideLane* side) {
#define FCH_COL(E_, P_) \
  if (epi == E_ && pro == P_) return lc<E_, P_>(a, s, e0, e1, side);
    FCH_COL(EPI_NONE, PRO_FIELD)
    FCH_COL(EPI_NONE, PRO_EXTRAP)
    FCH_COL(EPI_NONE, PRO_PSD_INIT)
    FCH_COL(EPI_MU, PRO_NONE)
    FCH_COL(EPI_F, PRO_NONE)
    FCH_COL(EPI_IMEX, PRO_NONE)
    FCH_COL(EPI_IMEX, PRO_NEXT_EXTRAP)
    FCH_COL(EPI_IMEX, PRO_NEXT_FIELD)
    FCH_COL(EPI_SAV, PRO_NONE)
    FCH_COL(EPI_PSD, PRO_NEXT_FIELD)
    FCH_COL(EPI_AM3, PRO_NONE)
    FCH_COL(EPI_NONE, PRO_ETD1)
    FCH_COL(EPI_NONE, PRO_SAV_NEXT)
    FCH_COL(EPI_ETD1, PRO_NEXT_FIELD)
    FCH_COL(EPI_ETD2, PRO_NEXT_FIELD)
    FCH_COL(EPI_ETD2, PRO_NONE)
#undef FCH_COL
    return hipErrorInvalidValue;
  }
  static hipError_t col_fwd1(const ColArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    FCH_LAUNCH((k_col1<N, E, -1, TWL>), dim3((H + 1) / 2), dim3(CT), s, e0, e1, a);
    return hipGetLastError();
  }
  static hipError_t col_inv1(const ColArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    FCH_LAUNCH((k_col1<N, E, +1, TWL>), dim3((H + 1) / 2), dim3(CT), s, e0, e1, a);
    return hipGetLastError();
  }
  static hipError_t col_ens(int stage, EnsMember* m, int first, int count, hipStream_t s) {
    const dim3 grid(N / 2, count);  // workgroup 0 takes both self-conjugate columns
    switch (stage) {
      case ENS_PRO:
        hipLaunchKernelGGL((k_col_ens<N, E, TWL, ENS_PRO>), grid, dim3(CT), 0, s, m, first);
        break;
      case ENS_IMEX:
        hipLaunchKernelGGL((k_col_ens<N, E, TWL, ENS_IMEX>), grid, dim3(CT), 0, s, m, first);
        break;
      case ENS_AM3:
        hipLaunchKernelGGL((k_col_ens<N, E, TWL, ENS_AM3>), grid, dim3(CT), 0, s, m, first);
        break;
      case ENS_ETD_PRO:
        hipLaunchKernelGGL((k_col_ens<N, E, TWL, ENS_ETD_PRO>), grid, dim3(CT), 0, s, m, first);
        break;
      case ENS_ETD2:
        hipLaunchKernelGGL((k_col_ens<N, E, TWL, ENS_ETD2>), grid, dim3(CT), 0, s, m, first);
        break;
      case ENS_SAV:
        hipLaunchKernelGGL((k_col_ens<N, E, TWL, ENS_SAV>), grid, dim3(CT), 0, s, m, first);
        break;
      case ENS_SAV_FIELD:
        hipLaunchKernelGGL((k_col_ens<N, E, TWL, ENS_SAV_FIELD>), grid, dim3(CT), 0, s, m, first);
        break;
      case ENS_PSD_INIT:
        hipLaunchKernelGGL((k_col_ens<N, E, TWL, ENS_PSD_INIT>), grid, dim3(CT), 0, s, m, first);
        break;
      case ENS_PSD:
        hipLaunchKernelGGL((k_col_ens<N, E, TWL, ENS_PSD>), grid, dim3(CT), 0, s, m, first);
        break;
      default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  static hipError_t col1_batch(int dir, const ColArgs& a, int batch, size_t sstride,
                               hipStream_t s) {
    const dim3 grid((H + 1) / 2, batch);
    if (dir < 0)
      hipLaunchKernelGGL((k_col1_b<N, E, -1, TWL>), grid, dim3(CT), 0, s, a, sstride);
    else
      hipLaunchKernelGGL((k_col1_b<N, E, +1, TWL>), grid, dim3(CT), 0, s, a, sstride);
    return hipGetLastError();
  }
  static const ColVT* table() {
    static const ColVT vt = {N, E, TWL, CT, &col, &col_fwd1, &col_inv1, &col_ens, &col1_batch};
    return &vt;
  }
};

template <int N, int R, int ER, int RTWL, int EC, int CTWL, int WPE>
struct PsdSolveImpl {
  static hipError_t launch(const RowArgs& ra, const ColArgs& ca, int limit, int grid,
                           hipStream_t s) {
    hipLaunchKernelGGL((k_psd_solve<N, R, ER, RTWL, EC, CTWL, WPE>), dim3(grid), dim3(N / EC), 0, s,
                       ra, ca, limit);
    return hipGetLastError();
  }
  static const PsdSolveVT* table() {
    static const PsdSolveVT vt = {N,    R,    ER,
                                  RTWL, EC,   CTWL,
                                  N / EC, (const void*)&k_psd_solve<N, R, ER, RTWL, EC, CTWL, WPE>,
                                  &launch};
    return &vt;
  }
};

}  // namespace fch

// The one-launch PSD solve of one grid size:
//   FCH_PSD_SOLVE(N, R, ER, RTWL, EC, CTWL, waves per SIMD of the launch bound)
#define FCH_PSD_SOLVE(N, R, ER, RTWL, EC, CTWL, WPE)                  \
  namespace fch {                                                     \
  const PsdSolveVT* psd_solve_##N() {                                 \
    return PsdSolveImpl<N, R, ER, RTWL, EC, CTWL, WPE>::table();      \
  }                                                                   \
  }

// Defines the variant lists of one grid size:
//   FCH_VARIANTS(N, (RowImpl<...>::table(), ...), (ColImpl<...>::table(), ...))
#define FCH_LIST(...) __VA_ARGS__
#define FCH_VARIANTS(N, ROWS, COLS)                                              \
  namespace fch {                                                                \
  const RowVT* const* row_variants_##N(int* n) {                                 \
    static const RowVT* const v[] = {ROWS};                                      \
    *n = (int)(sizeof(v) / sizeof(v[0]));                                        \
    return v;                                                                    \
  }                                                                              \
  const ColVT* const* col_variants_##N(int* n) {                                 \
    static const ColVT* const v[] = {COLS};                                      \
    *n = (int)(sizeof(v) / sizeof(v[0]));                                        \
    return v;                                                                    \
  }                                                                              \
  }
