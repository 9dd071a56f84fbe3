// Launches of mb4_spectral.hip used by the runtime.
#pragma once

#include "mb4_internal.h"

namespace mb4 {

// Spectrally preconditioned stage solves (mb4_spectral.hip), for kinetic
// operators too stiff for block-Jacobi sweeps.  Line-DFT passes over the
// three stage systems: pass 0 (rows) forms -Phibar (rbar = 0) and transforms
// it into io; pass 1 (columns) transforms, applies M^{-1} and transforms
// back; pass 2 (rows) transforms back into the new rbar in r, forms the next
// right-hand side -Phibar - D rbar (D = A - M, the site-local part of the
// stage matrix A that the preconditioner M leaves out) and transforms it;
// pass 3 (rows) is pass 2 without the next right-hand side.  So K Richardson
// iterations are pass 0, then (1, 2) K - 1 times, then (1, 3).  Pass 2 and 3
// post ||(T (x) I) rbar||_inf to *rslot if not NULL.  Every launch returns
// at once when `check` holds.  Sides up to kMaxSpectralSide.
constexpr int kMaxSpectralSide = 1024;

struct SpectralArgs {
  double kappa0;       // V_ref + shift: the preconditioner's on-site value
  const double2* twx;  // e^{-2 pi i m / nx}, m = 0 .. nx-1 (device)
  const double2* twy;  // e^{-2 pi i m / ny}, m = 0 .. ny-1 (device)
};

hipError_t launch_spectral_pass(int pass, const Lattice& lat, CPlanes3 phib, Planes3 io,
                                Planes3 r, const SpectralArgs& sa, unsigned long long* rslot,
                                ConvCheck check, hipStream_t stream, LaunchEvents ev = {});

}  // namespace mb4
