// Spectrally preconditioned stage solves, for kinetic operators too stiff
// for block-Jacobi sweeps: the continuum -Delta_h of Sec. 3 (hopping
// t = 1/h_x^2, diagonal shift 4 t) makes h lambda_i t reach ~10 per link,
// where the sweeps of k_stage_solve diverge.
//
// The stage system of Eq. MB4_5, A_i rbar_i = -Phibar_i with
// A_i = I - h lambda_i J, is solved by preconditioned Richardson iterations
// with M_i the constant-coefficient part of A_i.  Written for psi = p + i q,
// S acts as multiplication by -i, so with K_c = V_ref + shift - t * (sum
// over the four neighbours), M_i psi = (1 + i h lambda_i K_c) psi, which the
// 2D discrete Fourier transform diagonalises: mode (kx, ky) is multiplied by
// 1 + i h lambda_i kappa, kappa = V_ref + shift - 2 t (cos(2 pi kx / nx)
// + cos(2 pi ky / ny)).  The rest, D_i = A_i - M_i, is a 2x2 block per site
// (the potential's deviation from V_ref and the cubic term's Jacobian), so
// the iteration
//   rbar <- rbar + M_i^{-1} (-Phibar_i - A_i rbar) = M_i^{-1} (-Phibar_i - D_i rbar)
// needs no stencil: its right-hand side is formed site by site as the first
// transform reads it.  |1 + i b| >= 1, so one iteration contracts the error
// by at most h lambda_i ||D_i||.
//
// The transforms are line DFTs done directly (O(n) per output, n <= 1024):
// one block per grid line holds the line of all three stages and the
// twiddles in LDS, so every pass works in place.  The column pass does the
// forward transform, M^{-1} and the inverse transform of its column; the row
// pass does the inverse transform of its row (the new rbar, and on the last
// iteration ||(T (x) I) rbar||_inf), then forms the next right-hand side and
// transforms it forward.  A Richardson iteration is therefore two launches.
#include <float.h>
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "mb4_constants.h"
#include "mb4_internal.h"
#include "mb4_spectral.h"

namespace mb4 {
namespace {

constexpr int kLineThreads = 512;

__device__ __forceinline__ unsigned long long abs_bits_s(double v) {
  return static_cast<unsigned long long>(__double_as_longlong(fabs(v)));
}

__device__ __forceinline__ bool converged_s(const ConvCheck& c) {
  if (c.rec == nullptr) return false;
  const double r = __longlong_as_double(static_cast<long long>(c.rec[c.prev]));
  double tol = c.eps;
  if (c.relative) {
    const double u0max = __longlong_as_double(static_cast<long long>(c.rec[0]));
    tol = c.eps * (u0max > DBL_MIN ? u0max : DBL_MIN);
  }
  return r <= tol;
}

using LineBuf = double2[3][kMaxSpectralSide];

// Output k of the length-n DFT of the line `in`, forward (e^{-2 pi i jk/n})
// or inverse (e^{+2 pi i jk/n}, unscaled); tw holds e^{-2 pi i m/n},
// m = 0 .. n-1.  Even and odd j go to separate sums.
__device__ __forceinline__ double2 line_dft(const double2* in, const double2* tw, int n, int k,
                                            bool inverse) {
  double ax0 = 0.0, ay0 = 0.0, ax1 = 0.0, ay1 = 0.0;
  int m = 0;  // j * k mod n
  int j = 0;
  for (; j + 1 < n; j += 2) {
    const double2 w0 = tw[m];
    m += k;
    if (m >= n) m -= n;
    const double2 w1 = tw[m];
    m += k;
    if (m >= n) m -= n;
    const double2 v0 = in[j], v1 = in[j + 1];
    const double wy0 = inverse ? -w0.y : w0.y, wy1 = inverse ? -w1.y : w1.y;
    ax0 += v0.x * w0.x - v0.y * wy0;
    ay0 += v0.x * wy0 + v0.y * w0.x;
    ax1 += v1.x * w1.x - v1.y * wy1;
    ay1 += v1.x * wy1 + v1.y * w1.x;
  }
  if (j < n) {
    const double2 w = tw[m];
    const double wy = inverse ? -w.y : w.y;
    const double2 v = in[j];
    ax0 += v.x * w.x - v.y * wy;
    ay0 += v.x * wy + v.y * w.x;
  }
  return make_double2(ax0 + ax1, ay0 + ay1);
}

// Block maximum of rm into *slot (u64 bit patterns of non-negative doubles;
// NaN patterns sort above +inf and survive).
__device__ void line_max_to(unsigned long long rm, unsigned long long* slot) {
  constexpr int kW = kLineThreads / 64;
  __shared__ unsigned long long red[kW];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long o = __shfl_xor(rm, off, 64);
    rm = o > rm ? o : rm;
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = rm;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long mx = red[0];
#pragma unroll
    for (int w = 1; w < kW; ++w) mx = red[w] > mx ? red[w] : mx;
    const unsigned long long cur =
        __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (mx > cur) atomicMax(slot, mx);
  }
}

// Row pass (one block per row y = blockIdx.x; each thread takes (output,
// stage) pairs).  INV: inverse DFT of the row of io, scaled by 1 / (nx ny),
// is the new rbar, stored to r (with ||(T (x) I) rbar||_inf to *rslot if not
// NULL and not FWD).  FWD: the right-hand side -Phibar - D rbar of the next
// Richardson iteration (-Phibar when not INV, i.e. rbar = 0) is formed site
// by site and its forward DFT goes to io.
template <bool INV, bool FWD>
__global__ __launch_bounds__(kLineThreads) void k_spec_rows(Lattice L, CPlanes3 phib, Planes3 io,
                                                            Planes3 r, SpectralArgs sa,
                                                            unsigned long long* rslot,
                                                            ConvCheck chk) {
  if (converged_s(chk)) return;
  const int nx = L.nx, ny = L.ny;
  const int row = blockIdx.x * nx;
  const int items = 3 * nx;
  __shared__ LineBuf a, b;
  __shared__ double2 stw[kMaxSpectralSide];
  for (int e = threadIdx.x; e < nx; e += kLineThreads) {
    stw[e] = sa.twx[e];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      if (INV) {
        a[i][e] = io.s[i][row + e];
      } else {
        const double2 ph = phib.s[i][row + e];
        a[i][e] = make_double2(-ph.x, -ph.y);
      }
    }
  }
  __syncthreads();
  if (INV) {
    const double scale = 1.0 / (double(nx) * double(ny));
    for (int w = threadIdx.x; w < items; w += kLineThreads) {
      const int i = w / nx, k = w - i * nx;
      const int site = row + k;
      double2 rv = line_dft(a[i], stw, nx, k, true);
      rv.x *= scale;
      rv.y *= scale;
      r.s[i][site] = rv;
      if (FWD) {
        // D_i = h lambda_i [[-ca, -db], [dc, ca]]: the site block of
        // Eqs. JL, JR less M's on-site part kappa0.
        const double2 u = L.u0[site];
        const double pp = u.x * u.x, qq = u.y * u.y;
        const double dv = (L.V[site] + L.shift) - sa.kappa0;
        const double g = L.gs != nullptr ? L.gs[site] : L.g;
        const double ca = 2.0 * g * u.x * u.y;
        const double db = dv + g * (pp + 3.0 * qq);
        const double dc = dv + g * (3.0 * pp + qq);
        const double hl = L.h * MB4_LAMBDA[i];
        const double2 ph = phib.s[i][site];
        b[i][k] = make_double2(-ph.x + hl * (ca * rv.x + db * rv.y),
                               -ph.y - hl * (dc * rv.x + ca * rv.y));
      } else {
        b[i][k] = rv;
      }
    }
    __syncthreads();
    if (!FWD && rslot != nullptr) {
      unsigned long long rm = 0ull;
      for (int k = threadIdx.x; k < nx; k += kLineThreads) {
        const double2 r0 = b[0][k], r1 = b[1][k], r2 = b[2][k];
#pragma unroll
        for (int mm = 0; mm < 3; ++mm) {
          const double dx = MB4_T[mm][0] * r0.x + MB4_T[mm][1] * r1.x + MB4_T[mm][2] * r2.x;
          const double dy = MB4_T[mm][0] * r0.y + MB4_T[mm][1] * r1.y + MB4_T[mm][2] * r2.y;
          const unsigned long long bx = abs_bits_s(dx), by = abs_bits_s(dy);
          rm = bx > rm ? bx : rm;
          rm = by > rm ? by : rm;
        }
      }
      line_max_to(rm, rslot);
    }
  }
  if (FWD) {
    const LineBuf& src = INV ? b : a;
    for (int w = threadIdx.x; w < items; w += kLineThreads) {
      const int i = w / nx, k = w - i * nx;
      io.s[i][row + k] = line_dft(src[i], stw, nx, k, false);
    }
  }
}

// Column pass (one block per column x = blockIdx.x; each thread takes
// (output, stage) pairs): forward DFT along y, multiplication of mode
// (kx, ky) = (x, k) by 1 / (1 + i h lambda_i kappa), inverse DFT along y, in
// place in io.
__global__ __launch_bounds__(kLineThreads) void k_spec_cols(Lattice L, Planes3 io, SpectralArgs sa,
                                                            ConvCheck chk) {
  if (converged_s(chk)) return;
  const int nx = L.nx, ny = L.ny;
  const int col = blockIdx.x;
  const int items = 3 * ny;
  __shared__ LineBuf a, b;
  __shared__ double2 stw[kMaxSpectralSide];
  for (int e = threadIdx.x; e < ny; e += kLineThreads) {
    stw[e] = sa.twy[e];
#pragma unroll
    for (int i = 0; i < 3; ++i) a[i][e] = io.s[i][e * nx + col];
  }
  __syncthreads();
  // cos(2 pi kx / nx) is the real part of the twiddle e^{-2 pi i kx / nx}.
  const double cx = sa.twx[col].x;
  for (int w = threadIdx.x; w < items; w += kLineThreads) {
    const int i = w / ny, k = w - i * ny;
    const double2 v = line_dft(a[i], stw, ny, k, false);
    const double kappa = sa.kappa0 - 2.0 * L.t * (cx + stw[k].x);
    const double bm = L.h * MB4_LAMBDA[i] * kappa;
    const double d = 1.0 / (1.0 + bm * bm);
    b[i][k] = make_double2((v.x + bm * v.y) * d, (v.y - bm * v.x) * d);
  }
  __syncthreads();
  for (int w = threadIdx.x; w < items; w += kLineThreads) {
    const int i = w / ny, k = w - i * ny;
    io.s[i][k * nx + col] = line_dft(b[i], stw, ny, k, true);
  }
}

}  // namespace

hipError_t launch_spectral_pass(int pass, const Lattice& lat, CPlanes3 phib, Planes3 io,
                                Planes3 r, const SpectralArgs& sa, unsigned long long* rslot,
                                ConvCheck check, hipStream_t stream, LaunchEvents ev) {
  if (lat.nx > kMaxSpectralSide || lat.ny > kMaxSpectralSide) return hipErrorInvalidValue;
  const dim3 block(kLineThreads);
  const bool timed = ev.start != nullptr || ev.stop != nullptr;
#define MB4_SPEC_ROWS(I, F)                                                                   \
  do {                                                                                        \
    const dim3 grid(lat.ny);                                                                  \
    if (!timed)                                                                               \
      hipLaunchKernelGGL((k_spec_rows<I, F>), grid, block, 0, stream, lat, phib, io, r, sa,   \
                         rslot, check);                                                       \
    else                                                                                      \
      hipExtLaunchKernelGGL((k_spec_rows<I, F>), grid, block, 0, stream, ev.start, ev.stop,  \
                            0u, lat, phib, io, r, sa, rslot, check);                          \
  } while (0)
  switch (pass) {
    case 0: MB4_SPEC_ROWS(false, true); break;
    case 1: {
      const dim3 grid(lat.nx);
      if (!timed)
        hipLaunchKernelGGL(k_spec_cols, grid, block, 0, stream, lat, io, sa, check);
      else
        hipExtLaunchKernelGGL(k_spec_cols, grid, block, 0, stream, ev.start, ev.stop, 0u, lat,
                              io, sa, check);
      break;
    }
    case 2: MB4_SPEC_ROWS(true, true); break;
    case 3: MB4_SPEC_ROWS(true, false); break;
    default: return hipErrorInvalidValue;
  }
#undef MB4_SPEC_ROWS
  return hipGetLastError();
}

}  // namespace mb4
