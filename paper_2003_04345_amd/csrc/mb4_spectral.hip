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
// one block per grid line, the line of all three stages and the twiddles in
// LDS.  Rows are transformed (their right-hand side formed on the way in),
// then columns with the mode multiplication fused in; the inverse runs rows,
// then columns, which store the new rbar (and on the last iteration reduce
// ||(T (x) I) rbar||_inf).  Every line is owned by one block, so the passes
// work in place.
#include <float.h>
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "mb4_constants.h"
#include "mb4_internal.h"

namespace mb4 {
namespace {

constexpr int kLineThreads = 256;

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

// One pass of line DFTs (see the file comment).  PASS 0: forward along x
// (rows) of -Phibar - D r (of -Phibar if `first`) into io; PASS 1: forward
// along y (columns) and multiplication by 1 / (1 + i h lambda_i kappa);
// PASS 2: inverse along x; PASS 3: inverse along y, scaled by 1 / (nx ny),
// into r, and the norm to *rslot if not NULL.
template <int PASS>
__global__ __launch_bounds__(kLineThreads) void k_spec_lines(Lattice L, CPlanes3 phib, Planes3 io,
                                                             Planes3 r, SpectralArgs sa,
                                                             int first,
                                                             unsigned long long* rslot,
                                                             ConvCheck chk) {
  if (converged_s(chk)) return;
  constexpr bool ALONG_X = PASS == 0 || PASS == 2;
  constexpr bool INVERSE = PASS >= 2;
  const int nx = L.nx, ny = L.ny;
  const int n = ALONG_X ? nx : ny;
  const int line = blockIdx.x;
  const double2* tw = ALONG_X ? sa.twx : sa.twy;
  __shared__ double2 buf[3][kMaxSpectralSide];
  __shared__ double2 stw[kMaxSpectralSide];
  auto site_of = [&](int e) { return ALONG_X ? line * nx + e : e * nx + line; };
  for (int e = threadIdx.x; e < n; e += kLineThreads) {
    const int site = site_of(e);
    stw[e] = tw[e];
    if (PASS == 0) {
      // D r with D = [[-hl a, -hl (b - kappa0)], [hl (c - kappa0), hl a]]:
      // the site block of Eqs. JL, JR less M's on-site part kappa0.
      double a = 0.0, db = 0.0, dc = 0.0;
      if (!first) {
        const double2 u = L.u0[site];
        const double pp = u.x * u.x, qq = u.y * u.y;
        const double dv = (L.V[site] + L.shift) - sa.kappa0;
        a = 2.0 * L.g * u.x * u.y;
        db = dv + L.g * (pp + 3.0 * qq);
        dc = dv + L.g * (3.0 * pp + qq);
      }
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const double2 ph = phib.s[i][site];
        double2 v = make_double2(-ph.x, -ph.y);
        if (!first) {
          const double hl = L.h * MB4_LAMBDA[i];
          const double2 ri = r.s[i][site];
          v.x -= -hl * (a * ri.x + db * ri.y);
          v.y -= hl * (dc * ri.x + a * ri.y);
        }
        buf[i][e] = v;
      }
    } else {
#pragma unroll
      for (int i = 0; i < 3; ++i) buf[i][e] = io.s[i][site];
    }
  }
  __syncthreads();
  unsigned long long rm = 0ull;
  for (int k = threadIdx.x; k < n; k += kLineThreads) {
    double2 acc[3] = {make_double2(0.0, 0.0), make_double2(0.0, 0.0), make_double2(0.0, 0.0)};
    int m = 0;  // j * k mod n
    for (int j = 0; j < n; ++j) {
      const double2 w = stw[m];
      const double wy = INVERSE ? -w.y : w.y;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const double2 v = buf[i][j];
        acc[i].x += v.x * w.x - v.y * wy;
        acc[i].y += v.x * wy + v.y * w.x;
      }
      m += k;
      if (m >= n) m -= n;
    }
    const int site = site_of(k);
    if (PASS == 1) {
      // Mode (kx, ky) = (line, k): cos(2 pi kx / nx) is the real part of
      // the twiddle e^{-2 pi i kx / nx}.
      const double kappa = sa.kappa0 - 2.0 * L.t * (sa.twx[line].x + stw[k].x);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const double b = L.h * MB4_LAMBDA[i] * kappa;
        const double d = 1.0 / (1.0 + b * b);
        const double2 v = acc[i];
        acc[i] = make_double2((v.x + b * v.y) * d, (v.y - b * v.x) * d);
      }
    }
    if (PASS < 3) {
#pragma unroll
      for (int i = 0; i < 3; ++i) io.s[i][site] = acc[i];
    } else {
      const double scale = 1.0 / (double(nx) * double(ny));
      double2 rv[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        rv[i] = make_double2(acc[i].x * scale, acc[i].y * scale);
        r.s[i][site] = rv[i];
      }
      if (rslot != nullptr) {
#pragma unroll
        for (int mm = 0; mm < 3; ++mm) {
          const double dx = MB4_T[mm][0] * rv[0].x + MB4_T[mm][1] * rv[1].x + MB4_T[mm][2] * rv[2].x;
          const double dy = MB4_T[mm][0] * rv[0].y + MB4_T[mm][1] * rv[1].y + MB4_T[mm][2] * rv[2].y;
          const unsigned long long bx = abs_bits_s(dx), by = abs_bits_s(dy);
          // NaN patterns sort above +inf and survive the maximum.
          rm = bx > rm ? bx : rm;
          rm = by > rm ? by : rm;
        }
      }
    }
  }
  if (PASS == 3 && rslot != nullptr) {
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
          __hip_atomic_load(rslot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (mx > cur) atomicMax(rslot, mx);
    }
  }
}

}  // namespace

hipError_t launch_spectral_pass(int pass, const Lattice& lat, CPlanes3 phib, Planes3 io,
                                Planes3 r, const SpectralArgs& sa, bool first,
                                unsigned long long* rslot, ConvCheck check, hipStream_t stream,
                                LaunchEvents ev) {
  if (lat.nx > kMaxSpectralSide || lat.ny > kMaxSpectralSide) return hipErrorInvalidValue;
  const bool along_x = pass == 0 || pass == 2;
  const dim3 grid(along_x ? lat.ny : lat.nx), block(kLineThreads);
  const int f = first ? 1 : 0;
#define MB4_SPEC_PASS(P)                                                                      \
  do {                                                                                        \
    if (ev.start == nullptr && ev.stop == nullptr)                                            \
      hipLaunchKernelGGL(k_spec_lines<P>, grid, block, 0, stream, lat, phib, io, r, sa, f,    \
                         rslot, check);                                                       \
    else                                                                                      \
      hipExtLaunchKernelGGL(k_spec_lines<P>, grid, block, 0, stream, ev.start, ev.stop, 0u,  \
                            lat, phib, io, r, sa, f, rslot, check);                          \
  } while (0)
  switch (pass) {
    case 0: MB4_SPEC_PASS(0); break;
    case 1: MB4_SPEC_PASS(1); break;
    case 2: MB4_SPEC_PASS(2); break;
    case 3: MB4_SPEC_PASS(3); break;
    default: return hipErrorInvalidValue;
  }
#undef MB4_SPEC_PASS
  return hipGetLastError();
}

}  // namespace mb4
