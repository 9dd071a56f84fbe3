// HIP kernels of one MB4 step on the periodic 2D lattice (gfx950, FP64).
//
// Method: Sakai et al., arXiv 2003.04345, Sec. 2.2-2.3 and Algorithm 1.
//  * k_first_residual:  transformed residual at the initial guess
//    U^0 = e_3 (x) u_0 (Algorithm 1, Newton loop entry).
//  * k_update_residual: U <- U + (T (x) I) rbar (Eq. MB4_6 and the update of
//    Eq. Newton1), the stage combinations and S grad H at the Gauss-Legendre
//    nodes (Eqs. Lagrange, fKu2, fIu2), Phi (Eq. Phidefinition), the
//    transform Phibar = (T^-1 (x) I) Phi (Eq. MB4_4) and ||r||_inf, in one
//    pass over LDS tiles with a one-site halo.
//  * k_stage_sweep: one block-Jacobi sweep for all three decoupled stage
//    systems (I - h lambda_i J) rbar_i = -Phibar_i (Eq. MB4_5) at once, with
//    J frozen at u_0 (Eqs. Jacobianall, JL, JR).
//  * k_energy_*: H and its parts (Sec. 2.1) by a fixed-order double-double
//    reduction.
//
// Layout: every field is an array of double2 (p, q) per site, site = y*nx+x;
// a stage field is three such planes.  Tiles of 64 x 4 sites (one 256-thread
// block, four wave64s); the block -> tile map is XCD-aware so that the tiles
// one XCD works on are contiguous and share halo rows in its L2.
#include <float.h>
#include <hip/hip_ext.h>

#include "mb4_constants.h"
#include "mb4_internal.h"

namespace mb4 {
namespace {

constexpr int kTX = 64;
constexpr int kTY = 4;
constexpr int kTile = kTX * kTY;
constexpr int kWaves = kTile / 64;
constexpr int kXcds = 8;
constexpr int kRing = 2 * (kTX + 2) + 2 * kTY;   // halo positions of a tile
static_assert(kRing <= kTile, "halo ring must fit one pass of the block");

__device__ __forceinline__ int wrap(int v, int n) {
  while (v >= n) v -= n;
  while (v < 0) v += n;
  return v;
}

// Workgroups are dispatched round-robin over the 8 XCDs.  Remap so that XCD
// k receives the k-th contiguous range of logical tiles.
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int q = nb / kXcds, r = nb % kXcds;
  const int x = b % kXcds, k = b / kXcds;
  return x * q + min(x, r) + k;
}

__device__ __forceinline__ unsigned long long abs_bits(double v) {
  // |v| as an ordered bit pattern; NaN patterns sort above +inf, so a NaN
  // survives an unsigned max and later fails every convergence test.
  return static_cast<unsigned long long>(__double_as_longlong(fabs(v)));
}

__device__ __forceinline__ unsigned long long umax(unsigned long long a, unsigned long long b) {
  return a > b ? a : b;
}

__device__ __forceinline__ double conv_tol(double eps, double u0max) {
  return eps * (u0max > DBL_MIN ? u0max : DBL_MIN);
}

__device__ __forceinline__ bool skip_iteration(const ConvCheck& c) {
  if (c.stats == nullptr) return false;
  const double u0max = __longlong_as_double(static_cast<long long>(c.stats->u0max));
  const double r = __longlong_as_double(static_cast<long long>(c.stats->rmax[c.prev]));
  return r <= conv_tol(c.eps, u0max);
}

// Block-wide max of v, then one atomic per block.
__device__ __forceinline__ void block_max_to(unsigned long long v, unsigned long long* slot) {
  __shared__ unsigned long long red[kWaves];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = umax(v, __shfl_xor(v, off, 64));
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long m = red[0];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) m = umax(m, red[w]);
    // Device-scope atomics on one address serialise across the XCDs; most
    // blocks hold a value below the running maximum, so read it first (a
    // coherent load) and only post a larger value.  The slot only grows, so a
    // block that skips has v <= what the slot already holds.
    const unsigned long long cur =
        __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (m > cur) atomicMax(slot, m);
  }
}

struct TileCoord {
  int x0, y0, x, y;
  bool inside;
};

__device__ __forceinline__ TileCoord tile_coord(int nx, int ny) {
  const int tiles_x = (nx + kTX - 1) / kTX;
  const int b = xcd_block(blockIdx.x, gridDim.x);
  TileCoord c;
  c.x0 = (b % tiles_x) * kTX;
  c.y0 = (b / tiles_x) * kTY;
  c.x = c.x0 + (threadIdx.x % kTX);
  c.y = c.y0 + (threadIdx.x / kTX);
  c.inside = c.x < nx && c.y < ny;
  return c;
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_reset_stats(Stats* stats, int upto) {
  for (int i = threadIdx.x; i <= upto; i += 64) stats->rmax[i] = 0ull;
  if (threadIdx.x == 0) stats->u0max = 0ull;
}

// ---------------------------------------------------------------------------
// At U = e_3 (x) u_0 every stage value and every Gauss node equals u_0 (the
// Lagrange basis sums to one), so int A_{c_m,z} f(U_z) dz = c_m f(u_0) and
// Phi_m = -h c_m f(u_0); Phibar_i = -h TC_i f(u_0) with TC = T^-1 c.
__global__ __launch_bounds__(kTile) void k_first_residual(Lattice L, Planes3 phib, Stats* stats) {
  const TileCoord c = tile_coord(L.nx, L.ny);
  unsigned long long m = 0ull;
  if (c.inside) {
    const int nx = L.nx, ny = L.ny;
    const int site = c.y * nx + c.x;
    const int xl = c.x == 0 ? nx - 1 : c.x - 1, xr = c.x == nx - 1 ? 0 : c.x + 1;
    const int yd = c.y == 0 ? ny - 1 : c.y - 1, yu = c.y == ny - 1 ? 0 : c.y + 1;
    const double2 u = L.u0[site];
    const double2 a = L.u0[c.y * nx + xl], b = L.u0[c.y * nx + xr];
    const double2 d = L.u0[yd * nx + c.x], e = L.u0[yu * nx + c.x];
    const double sp = (a.x + b.x) + (d.x + e.x);
    const double sq = (a.y + b.y) + (d.y + e.y);
    const double vs = L.V[site] + L.shift;
    const double gn = L.g * (u.x * u.x + u.y * u.y);
    // f = S grad H = (A q + g n q, -(A p + g n p))
    const double fp = -L.t * sq + (vs + gn) * u.y;
    const double fq = L.t * sp - (vs + gn) * u.x;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double k = -L.h * MB4_TC[i];
      phib.s[i][site] = make_double2(k * fp, k * fq);
    }
    m = umax(abs_bits(u.x), abs_bits(u.y));
  }
  block_max_to(m, &stats->u0max);
}

// ---------------------------------------------------------------------------
// Updated stage values and their linear combinations W_i = E_i0 u_0 +
// sum_j E_ij U_j (Eq. fKu2) at one site.
template <bool FROM_U0, bool HAS_RBAR>
__device__ __forceinline__ void site_update(const Lattice& L, const CPlanes3& Uin,
                                            const CPlanes3& rb, int site, double2& u0,
                                            double2 (&Un)[3], double2 (&W)[3],
                                            unsigned long long& rm) {
  u0 = L.u0[site];
#pragma unroll
  for (int j = 0; j < 3; ++j) Un[j] = FROM_U0 ? u0 : Uin.s[j][site];
  rm = 0ull;
  if (HAS_RBAR) {
    double2 r[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) r[m] = rb.s[m][site];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const double dp = MB4_T[j][0] * r[0].x + MB4_T[j][1] * r[1].x + MB4_T[j][2] * r[2].x;
      const double dq = MB4_T[j][0] * r[0].y + MB4_T[j][1] * r[1].y + MB4_T[j][2] * r[2].y;
      Un[j].x += dp;
      Un[j].y += dq;
      rm = umax(rm, umax(abs_bits(dp), abs_bits(dq)));
    }
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    W[i].x = MB4_E0[i] * u0.x + MB4_E[i][0] * Un[0].x + MB4_E[i][1] * Un[1].x +
             MB4_E[i][2] * Un[2].x;
    W[i].y = MB4_E0[i] * u0.y + MB4_E[i][0] * Un[0].y + MB4_E[i][1] * Un[1].y +
             MB4_E[i][2] * Un[2].y;
  }
}

template <bool FROM_U0, bool HAS_RBAR>
__global__ __launch_bounds__(kTile) void k_update_residual(Lattice L, CPlanes3 Uin, Planes3 Uout,
                                                           CPlanes3 rb, Planes3 phib,
                                                           unsigned long long* rslot,
                                                           ConvCheck chk) {
  if (skip_iteration(chk)) return;
  __shared__ double2 sw[3][kTY + 2][kTX + 2];
  const int nx = L.nx, ny = L.ny;
  const TileCoord c = tile_coord(nx, ny);
  const int lx = threadIdx.x % kTX, ly = threadIdx.x / kTX;

  // Own position (wrapped when the tile overhangs the lattice: such a
  // position may still be the periodic neighbour of an inside site).
  const int gx = c.inside ? c.x : wrap(c.x, nx);
  const int gy = c.inside ? c.y : wrap(c.y, ny);
  const int site = gy * nx + gx;
  double2 u0, Un[3], W[3];
  unsigned long long rm;
  site_update<FROM_U0, HAS_RBAR>(L, Uin, rb, site, u0, Un, W, rm);
#pragma unroll
  for (int i = 0; i < 3; ++i) sw[i][ly + 1][lx + 1] = W[i];

  if (threadIdx.x < kRing) {
    const int k = threadIdx.x;
    int hx, hy;
    if (k < kTX + 2) {
      hx = k;
      hy = 0;
    } else if (k < 2 * (kTX + 2)) {
      hx = k - (kTX + 2);
      hy = kTY + 1;
    } else if (k < 2 * (kTX + 2) + kTY) {
      hx = 0;
      hy = 1 + k - 2 * (kTX + 2);
    } else {
      hx = kTX + 1;
      hy = 1 + k - 2 * (kTX + 2) - kTY;
    }
    const int hs = wrap(c.y0 + hy - 1, ny) * nx + wrap(c.x0 + hx - 1, nx);
    double2 hu0, hUn[3], hW[3];
    unsigned long long hrm;
    site_update<FROM_U0, HAS_RBAR>(L, Uin, rb, hs, hu0, hUn, hW, hrm);
#pragma unroll
    for (int i = 0; i < 3; ++i) sw[i][hy][hx] = hW[i];
  }
  __syncthreads();

  if (c.inside) {
    const double t = L.t, g = L.g, h = L.h;
    const double vs = L.V[site] + L.shift;
    double2 phi[3];
    // Linear part: int A_{c_i,z} (f_K + f_E)(U_z) dz = S A W_i (Eq. fKu2).
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double2 l = sw[i][ly + 1][lx], r = sw[i][ly + 1][lx + 2];
      const double2 d = sw[i][ly][lx + 1], u = sw[i][ly + 2][lx + 1];
      const double sp = (l.x + r.x) + (d.x + u.x);
      const double sq = (l.y + r.y) + (d.y + u.y);
      const double awp = -t * sp + vs * W[i].x;
      const double awq = -t * sq + vs * W[i].y;
      phi[i] = make_double2(awq, -awp);
    }
    // Cubic part (Eq. fIu2) by 6-node Gauss-Legendre, exact for degree 11.
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const double zp = MB4_GL_L[q][0] * u0.x + MB4_GL_L[q][1] * Un[0].x +
                        MB4_GL_L[q][2] * Un[1].x + MB4_GL_L[q][3] * Un[2].x;
      const double zq = MB4_GL_L[q][0] * u0.y + MB4_GL_L[q][1] * Un[0].y +
                        MB4_GL_L[q][2] * Un[1].y + MB4_GL_L[q][3] * Un[2].y;
      const double gn = g * (zp * zp + zq * zq);
      const double fp = gn * zq, fq = -gn * zp;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        phi[i].x += MB4_GL_Q[i][q] * fp;
        phi[i].y += MB4_GL_Q[i][q] * fq;
      }
    }
    // Phi_i = U_i - u_0 - h int A_{c_i,z} f(U_z) dz (Eq. Phidefinition).
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      phi[i].x = (Un[i].x - u0.x) - h * phi[i].x;
      phi[i].y = (Un[i].y - u0.y) - h * phi[i].y;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double bp = MB4_TINV[i][0] * phi[0].x + MB4_TINV[i][1] * phi[1].x +
                        MB4_TINV[i][2] * phi[2].x;
      const double bq = MB4_TINV[i][0] * phi[0].y + MB4_TINV[i][1] * phi[1].y +
                        MB4_TINV[i][2] * phi[2].y;
      phib.s[i][site] = make_double2(bp, bq);
      if (FROM_U0 || HAS_RBAR) Uout.s[i][site] = Un[i];
    }
  } else {
    rm = 0ull;
  }
  if (rslot != nullptr) block_max_to(rm, rslot);
}

// ---------------------------------------------------------------------------
// (I - h lambda_i J) r_i = b_i with b_i = -Phibar_i.  Per site the 2x2 block
// I - h lambda_i J_site, J_site = [[a, bb], [-cc, -a]] with a = 2 g p q,
// bb = A_jj + g (p^2 + 3 q^2), cc = A_jj + g (3 p^2 + q^2) (Eqs. JL, JR), is
// inverted exactly (its determinant is 1 + (h lambda)^2 (bb cc - a^2)); the
// hopping part of J couples neighbours through h lambda_i t (sum r_q,
// -sum r_p), which the sweep takes from the previous iterate.
template <bool FIRST>
__global__ __launch_bounds__(kTile) void k_stage_sweep(Lattice L, CPlanes3 phib, CPlanes3 rin,
                                                       Planes3 rout, ConvCheck chk) {
  if (skip_iteration(chk)) return;
  const int nx = L.nx, ny = L.ny;
  const TileCoord c = tile_coord(nx, ny);
  if (!c.inside) return;
  const int site = c.y * nx + c.x;
  const double2 u = L.u0[site];
  const double vs = L.V[site] + L.shift;
  const double g = L.g;
  const double pp = u.x * u.x, qq = u.y * u.y;
  const double a = 2.0 * g * u.x * u.y;
  const double bb = vs + g * (pp + 3.0 * qq);
  const double cc = vs + g * (3.0 * pp + qq);
  const double bc_a2 = bb * cc - a * a;
  int sl = 0, sr = 0, sd = 0, su = 0;
  if (!FIRST) {
    const int xl = c.x == 0 ? nx - 1 : c.x - 1, xr = c.x == nx - 1 ? 0 : c.x + 1;
    const int yd = c.y == 0 ? ny - 1 : c.y - 1, yu = c.y == ny - 1 ? 0 : c.y + 1;
    sl = c.y * nx + xl;
    sr = c.y * nx + xr;
    sd = yd * nx + c.x;
    su = yu * nx + c.x;
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double hl = L.h * MB4_LAMBDA[i];
    const double2 ph = phib.s[i][site];
    double bp = -ph.x, bq = -ph.y;
    if (!FIRST) {
      const double2 r1 = rin.s[i][sl], r2 = rin.s[i][sr], r3 = rin.s[i][sd], r4 = rin.s[i][su];
      const double sp = (r1.x + r2.x) + (r3.x + r4.x);
      const double sq = (r1.y + r2.y) + (r3.y + r4.y);
      const double ht = hl * L.t;
      bp -= ht * sq;
      bq += ht * sp;
    }
    const double inv = 1.0 / (1.0 + hl * hl * bc_a2);
    const double rp = inv * ((1.0 + hl * a) * bp + hl * bb * bq);
    const double rq = inv * ((1.0 - hl * a) * bq - hl * cc * bp);
    rout.s[i][site] = make_double2(rp, rq);
  }
}

// ---------------------------------------------------------------------------
// Double-double accumulation: TwoSum (Knuth) followed by renormalisation.
struct DD {
  double hi, lo;
};

__device__ __forceinline__ DD dd_add(DD a, DD b) {
  const double s = a.hi + b.hi;
  const double bb = s - a.hi;
  double e = (a.hi - (s - bb)) + (b.hi - bb);
  e += a.lo + b.lo;
  const double hi = s + e;
  return DD{hi, e - (hi - s)};
}

constexpr int kEnergyParts = 6;

// Per-block sums of the six energy terms; partials[(block*6 + k)*2 + {0,1}].
__global__ __launch_bounds__(kTile) void k_energy_partial(Lattice L, double* partials) {
  __shared__ DD red[kEnergyParts][kTile];
  const int nx = L.nx, ny = L.ny;
  const TileCoord c = tile_coord(nx, ny);
  double v[kEnergyParts] = {0, 0, 0, 0, 0, 0};
  if (c.inside) {
    const int site = c.y * nx + c.x;
    const int xl = c.x == 0 ? nx - 1 : c.x - 1, xr = c.x == nx - 1 ? 0 : c.x + 1;
    const int yd = c.y == 0 ? ny - 1 : c.y - 1, yu = c.y == ny - 1 ? 0 : c.y + 1;
    const double2 u = L.u0[site];
    const double2 a = L.u0[c.y * nx + xl], b = L.u0[c.y * nx + xr];
    const double2 d = L.u0[yd * nx + c.x], e = L.u0[yu * nx + c.x];
    const double sp = (a.x + b.x) + (d.x + e.x);
    const double sq = (a.y + b.y) + (d.y + e.y);
    const double n = u.x * u.x + u.y * u.y;
    const double uk = 0.5 * (L.shift * n - L.t * (u.x * sp + u.y * sq));
    const double ue = 0.5 * L.V[site] * n;
    const double ui = 0.25 * L.g * n * n;
    v[0] = uk + ue + ui;
    v[1] = uk;
    v[2] = ui;
    v[3] = ue;
    v[4] = n;
    v[5] = n * n;
  }
#pragma unroll
  for (int k = 0; k < kEnergyParts; ++k) red[k][threadIdx.x] = DD{v[k], 0.0};
  __syncthreads();
  for (int span = kTile / 2; span > 0; span >>= 1) {
    if (threadIdx.x < span) {
#pragma unroll
      for (int k = 0; k < kEnergyParts; ++k)
        red[k][threadIdx.x] = dd_add(red[k][threadIdx.x], red[k][threadIdx.x + span]);
    }
    __syncthreads();
  }
  if (threadIdx.x < kEnergyParts) {
    const DD s = red[threadIdx.x][0];
    partials[(static_cast<size_t>(blockIdx.x) * kEnergyParts + threadIdx.x) * 2 + 0] = s.hi;
    partials[(static_cast<size_t>(blockIdx.x) * kEnergyParts + threadIdx.x) * 2 + 1] = s.lo;
  }
}

__global__ __launch_bounds__(kTile) void k_energy_final(const double* partials, int nblocks,
                                                         double* out) {
  __shared__ DD red[kEnergyParts][kTile];
  DD acc[kEnergyParts];
#pragma unroll
  for (int k = 0; k < kEnergyParts; ++k) acc[k] = DD{0.0, 0.0};
  for (int bkt = threadIdx.x; bkt < nblocks; bkt += kTile) {
#pragma unroll
    for (int k = 0; k < kEnergyParts; ++k) {
      const size_t o = (static_cast<size_t>(bkt) * kEnergyParts + k) * 2;
      acc[k] = dd_add(acc[k], DD{partials[o], partials[o + 1]});
    }
  }
#pragma unroll
  for (int k = 0; k < kEnergyParts; ++k) red[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int span = kTile / 2; span > 0; span >>= 1) {
    if (threadIdx.x < span) {
#pragma unroll
      for (int k = 0; k < kEnergyParts; ++k)
        red[k][threadIdx.x] = dd_add(red[k][threadIdx.x], red[k][threadIdx.x + span]);
    }
    __syncthreads();
  }
  if (threadIdx.x < kEnergyParts) out[threadIdx.x] = red[threadIdx.x][0].hi + red[threadIdx.x][0].lo;
}

__global__ __launch_bounds__(256) void k_interleave(const double* p, const double* q, double2* out,
                                                    int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) out[i] = make_double2(p[i], q[i]);
}

__global__ __launch_bounds__(256) void k_deinterleave(const double2* in, double* p, double* q,
                                                      int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) {
    const double2 v = in[i];
    p[i] = v.x;
    q[i] = v.y;
  }
}

int tile_blocks(int nx, int ny) {
  return ((nx + kTX - 1) / kTX) * ((ny + kTY - 1) / kTY);
}

}  // namespace

// ---------------------------------------------------------------------------
// Every launch goes through hipExtLaunchKernelGGL so that, when the runtime
// asks for timing, the start/stop timestamps are taken by the dispatch itself
// (no extra marker packets between kernels).
#define MB4_LAUNCH(kernel, grid, block, ev, ...)                                             \
  do {                                                                                       \
    hipExtLaunchKernelGGL(kernel, grid, block, 0, stream, (ev).start, (ev).stop, 0u,        \
                          __VA_ARGS__);                                                      \
    return hipGetLastError();                                                                \
  } while (0)

hipError_t launch_reset_stats(Stats* stats, int upto, hipStream_t stream) {
  MB4_LAUNCH(k_reset_stats, dim3(1), dim3(64), LaunchEvents{}, stats, upto);
}

hipError_t launch_first_residual(const Lattice& lat, Planes3 phib, Stats* stats,
                                 hipStream_t stream, LaunchEvents ev) {
  MB4_LAUNCH(k_first_residual, dim3(tile_blocks(lat.nx, lat.ny)), dim3(kTile), ev, lat, phib,
             stats);
}

hipError_t launch_update_residual(const Lattice& lat, CPlanes3 Uin, Planes3 Uout, CPlanes3 rbar,
                                  bool has_rbar, bool from_u0, Planes3 phib,
                                  unsigned long long* rslot, ConvCheck check, hipStream_t stream,
                                  LaunchEvents ev) {
  const dim3 grid(tile_blocks(lat.nx, lat.ny)), block(kTile);
  if (from_u0 && has_rbar)
    MB4_LAUNCH((k_update_residual<true, true>), grid, block, ev, lat, Uin, Uout, rbar, phib,
               rslot, check);
  else if (from_u0)
    MB4_LAUNCH((k_update_residual<true, false>), grid, block, ev, lat, Uin, Uout, rbar, phib,
               rslot, check);
  else if (has_rbar)
    MB4_LAUNCH((k_update_residual<false, true>), grid, block, ev, lat, Uin, Uout, rbar, phib,
               rslot, check);
  else
    MB4_LAUNCH((k_update_residual<false, false>), grid, block, ev, lat, Uin, Uout, rbar, phib,
               rslot, check);
}

hipError_t launch_stage_sweep(const Lattice& lat, CPlanes3 phib, CPlanes3 rin, Planes3 rout,
                              bool first, ConvCheck check, hipStream_t stream, LaunchEvents ev) {
  const dim3 grid(tile_blocks(lat.nx, lat.ny)), block(kTile);
  if (first)
    MB4_LAUNCH(k_stage_sweep<true>, grid, block, ev, lat, phib, rin, rout, check);
  else
    MB4_LAUNCH(k_stage_sweep<false>, grid, block, ev, lat, phib, rin, rout, check);
}

hipError_t launch_interleave(const double* p, const double* q, double2* out, int n,
                             hipStream_t stream) {
  MB4_LAUNCH(k_interleave, dim3((n + 255) / 256), dim3(256), LaunchEvents{}, p, q, out, n);
}

hipError_t launch_deinterleave(const double2* in, double* p, double* q, int n,
                               hipStream_t stream) {
  MB4_LAUNCH(k_deinterleave, dim3((n + 255) / 256), dim3(256), LaunchEvents{}, in, p, q, n);
}

size_t energy_partials_count(int nx, int ny) {
  return static_cast<size_t>(tile_blocks(nx, ny)) * kEnergyParts * 2;
}

hipError_t launch_energy(const Lattice& lat, double* partials, double* out, hipStream_t stream) {
  const int nb = tile_blocks(lat.nx, lat.ny);
  hipExtLaunchKernelGGL(k_energy_partial, dim3(nb), dim3(kTile), 0, stream, nullptr, nullptr, 0u,
                        lat, partials);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipExtLaunchKernelGGL(k_energy_final, dim3(1), dim3(kTile), 0, stream, nullptr, nullptr, 0u,
                        static_cast<const double*>(partials), nb, out);
  return hipGetLastError();
}

}  // namespace mb4
