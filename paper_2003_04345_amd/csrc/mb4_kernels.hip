// HIP kernels of one MB4 step on the periodic 2D lattice (gfx950, FP64).
//
// Method: Sakai et al., arXiv 2003.04345, Sec. 2.2-2.3 and Algorithm 1.  One
// Newton iteration l is two passes over HBM:
//  * k_stage_solve: the three decoupled stage systems
//    (I - h lambda_i J) rbar_i = -Phibar_i (Eq. MB4_5), J frozen at u_0
//    (Eqs. Jacobianall, JL, JR), all three stages at once, by up to four
//    block-Jacobi sweeps temporally blocked in LDS; it also reduces
//    ||r||_inf = ||(T (x) I) rbar||_inf, the convergence measure of
//    Algorithm 1.  In iteration 1 it builds Phibar itself from u_0: at
//    U^0 = e_3 (x) u_0 the residual is Phi_m = -h c_m f(u_0).
//  * k_update_residual: if ||r^l||_inf met the tolerance, the accepted value
//    u_1 = U_{c_3} = U_3 + (T rbar)_3 is written over u_0 (Sec. 2.2: c_3 = 1)
//    and the step is done; otherwise U <- U + (T (x) I) rbar (Eqs. MB4_6,
//    Newton1), the stage combinations and S grad H at the Gauss-Legendre
//    nodes (Eqs. Lagrange, fKu2, fIu2), Phi (Eq. Phidefinition) and
//    Phibar = (T^-1 (x) I) Phi (Eq. MB4_4), over LDS tiles with a one-site
//    halo.
//  * k_stage_sweep: one more sweep, for solves that ask for more than four.
//  * k_energy_*: H and its parts (Sec. 2.1) by a fixed-order double-double
//    reduction.
//
// Layout: every field is an array of double2 (p, q) per site, site = y*nx+x;
// a stage field is three such planes.  Block -> tile maps are XCD-aware so
// that the tiles one XCD works on are contiguous and share halo rows in its
// L2.
#include <float.h>
#include <hip/hip_ext.h>

#include <algorithm>

#include "mb4_constants.h"
#include "mb4_internal.h"

namespace mb4 {
namespace {

constexpr int kTX = 64;
constexpr int kTY = 4;
constexpr int kTile = kTX * kTY;
constexpr int kXcds = 8;
constexpr int kRing = 2 * (kTX + 2) + 2 * kTY;   // halo positions of a residual tile
static_assert(kRing <= kTile, "halo ring must fit one pass of the block");

__device__ __forceinline__ int wrap(int v, int n) {
  while (v >= n) v -= n;
  while (v < 0) v += n;
  return v;
}

// The same for v in [-n, 2n) (a region on a lattice at least as wide as the
// region), without loops; `fast` (uniform) says whether that holds.
__device__ __forceinline__ int wrap_in(int v, int n, bool fast) {
  if (!fast) return wrap(v, n);
  v = v < 0 ? v + n : v;
  return v >= n ? v - n : v;
}

// Workgroups are dispatched round-robin over the 8 XCDs.  Remap so that XCD
// k receives the k-th contiguous range of logical tiles.
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int q = nb / kXcds, r = nb % kXcds;
  const int x = b % kXcds, k = b / kXcds;
  return x * q + min(x, r) + k;
}

// Tile (tx, ty) of block b (after xcd_block) on a tiles_x x tiles_y grid,
// walked in vertical strips kStrip tiles wide, row by row inside a strip.
// The blocks in flight on one XCD then hold vertically as well as
// horizontally adjacent tiles, so the halo rows a tile shares with the one
// above are still in that XCD's L2 (a row-major walk over a wide lattice
// has moved on by a whole tile row before they are read again).
constexpr int kStrip = 16;
__device__ __forceinline__ void strip_tile(int b, int tiles_x, int tiles_y, int& tx, int& ty) {
  const int full = tiles_x / kStrip;
  const int per = kStrip * tiles_y;
  if (b < full * per) {
    const int r = b % per;
    tx = (b / per) * kStrip + r % kStrip;
    ty = r / kStrip;
  } else {
    const int w = tiles_x - full * kStrip;
    const int r = b - full * per;
    tx = full * kStrip + r % w;
    ty = r / w;
  }
}

__device__ __forceinline__ unsigned long long abs_bits(double v) {
  // |v| as an ordered bit pattern; NaN patterns sort above +inf, so a NaN
  // survives an unsigned max and later fails every convergence test.
  return static_cast<unsigned long long>(__double_as_longlong(fabs(v)));
}

__device__ __forceinline__ unsigned long long umax(unsigned long long a, unsigned long long b) {
  return a > b ? a : b;
}

// Running max of |x| that keeps non-finite values.  The max is a plain FP64
// max, which skips a NaN, so the sum of the same values (NaN if any was) rides
// along; bits() is the IEEE pattern of the max, or of a NaN, which sorts
// above +inf in the unsigned block and device maxima.
struct NormAcc {
  double m = 0.0, s = 0.0;
  __device__ __forceinline__ void add(double x) {
    m = fmax(m, fabs(x));
    s += x;
  }
  __device__ __forceinline__ unsigned long long bits() const {
    return s != s ? 0x7ff8000000000000ull : abs_bits(m);
  }
};

__device__ __forceinline__ double bits_double(unsigned long long b) {
  return __longlong_as_double(static_cast<long long>(b));
}

__device__ __forceinline__ double conv_tol(double eps, double u0max) {
  return eps * (u0max > DBL_MIN ? u0max : DBL_MIN);
}

// True when Newton iteration c.prev (>= 1) already met the tolerance.  The
// record is read with a scalar load (it is not written while a kernel that
// tests it runs), which later blocks on a CU find in the scalar cache.
__device__ __forceinline__ bool converged_at(const ConvCheck& c) {
  if (c.rec == nullptr) return false;
  const double r = bits_double(c.rec[c.prev]);
  return r <= (c.relative ? conv_tol(c.eps, bits_double(c.rec[0])) : c.eps);
}

// The nonlinearity g at a site: its own g_j, or the lattice's g.
__device__ __forceinline__ double site_g(const Lattice& L, int site) {
  return L.gs != nullptr ? L.gs[site] : L.g;
}

// Where block b (after xcd_block) works: for a Multi, its member's lattice
// replaces L (with V and u0 moved to the member's sites), b becomes the block
// index within the member, and `base` / `rec` are the member's site and
// record offsets.  `skip`: the member takes no more steps in this batch.
struct Loc {
  int b, m;
  long long base, rec;
  bool skip;
};

// The member whose blocks [block0[m], block0[m + 1]) hold block b.
__device__ __forceinline__ int member_search(const int* block0, int count, int b) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (block0[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ Loc locate(const Multi& mu, Lattice& L, int b) {
  Loc w{b, 0, 0, 0, false};
  if (mu.desc == nullptr) return w;
  const int lo = mu.member_of != nullptr ? mu.member_of[b] : member_search(mu.block0, mu.count, b);
  const MemberDesc d = mu.desc[lo];
  w.b = b - mu.block0[lo];
  w.m = lo;
  w.base = d.base;
  w.rec = static_cast<long long>(lo) * mu.rec_stride;
  w.skip = mu.todo != nullptr && mu.step >= mu.todo[lo];
  L.nx = d.nx;
  L.ny = d.ny;
  L.t = d.t;
  L.shift = d.shift;
  L.g = d.g;
  L.h = d.h;
  L.V += d.base;
  L.u0 += d.base;
  if (L.gs != nullptr) L.gs += d.base;
  return w;
}

template <class P>
__device__ __forceinline__ void offset_planes(P& p, long long base) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
    if (p.s[i] != nullptr) p.s[i] += base;
}

__device__ __forceinline__ void offset_check(ConvCheck& c, long long rec) {
  if (c.rec != nullptr) c.rec += rec;
}

template <class T>
__device__ __forceinline__ T* offset_ptr(T* p, long long n) {
  return p == nullptr ? p : p + n;
}

// threadIdx.x through an empty asm statement, so that the compiler cannot
// hoist what a tile body derives from it out of a loop over tiles
// (k_member_run), where it would stay live, and spill, across the loop.
__device__ __forceinline__ int thread_index() {
  int t = static_cast<int>(threadIdx.x);
  asm volatile("" : "+v"(t));
  return t;
}

// Block-wide max of v posted to *slot.  Device-scope atomics on one address
// serialise across the XCDs; most blocks hold a value below the running
// maximum, so thread 0 reads it first (a coherent load) and only posts a
// larger value.  The slot only grows, so a block that skips has v <= what
// the slot already holds.  (Reading the slot earlier, when the block starts,
// lets more blocks post and is slower.)
template <int NT>
__device__ __forceinline__ void block_max_to(unsigned long long v, unsigned long long* slot) {
  constexpr int kW = NT / 64;
  __shared__ unsigned long long red[kW];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = umax(v, __shfl_xor(v, off, 64));
  __syncthreads();  // red[] may still be read by a previous reduction
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long m = red[0];
#pragma unroll
    for (int w = 1; w < kW; ++w) m = umax(m, red[w]);
    const unsigned long long cur =
        __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (m > cur) atomicMax(slot, m);
  }
}

struct TileCoord {
  int x0, y0, x, y;
  bool inside;
};

__device__ __forceinline__ TileCoord tile_coord_at(int nx, int ny, int b) {
  const int tiles_x = (nx + kTX - 1) / kTX;
  TileCoord c;
  c.x0 = (b % tiles_x) * kTX;
  c.y0 = (b / tiles_x) * kTY;
  c.x = c.x0 + (threadIdx.x % kTX);
  c.y = c.y0 + (threadIdx.x / kTX);
  c.inside = c.x < nx && c.y < ny;
  return c;
}

__device__ __forceinline__ TileCoord tile_coord(int nx, int ny) {
  return tile_coord_at(nx, ny, xcd_block(blockIdx.x, gridDim.x));
}

// r = (T (x) I) rbar at one site, component of stage j.
__device__ __forceinline__ double2 t_apply(int j, const double2 (&r)[3]) {
  return make_double2(MB4_T[j][0] * r[0].x + MB4_T[j][1] * r[1].x + MB4_T[j][2] * r[2].x,
                      MB4_T[j][0] * r[0].y + MB4_T[j][1] * r[1].y + MB4_T[j][2] * r[2].y);
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_clear_u64(unsigned long long* p, int n) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) p[i] = 0ull;
}

__global__ __launch_bounds__(256) void k_member_table(const int* block0, int count, int blocks,
                                                      int* member_of) {
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b < blocks) member_of[b] = member_search(block0, count, b);
}

// ---------------------------------------------------------------------------
// Updated stage values and their linear combinations W_i = E_i0 u_0 +
// sum_j E_ij U_j (Eq. fKu2) at one site.
// The iterate at one site after the update of this pass, and the linear
// stage combinations W_i (Eq. fKu2).  XFORM: the stage fields hold X = U -
// e (x) u_0 (Un receives X, and W_i = c_i u_0 + sum_j E_ij X_j, the full rows
// of E summing to c_i), which keeps the rounding of stored U out of W;
// otherwise they hold U.
template <bool FROM_U0, bool HAS_RBAR, bool XFORM>
__device__ __forceinline__ void site_update(const Lattice& L, const CPlanes3& Uin,
                                            const CPlanes3& rb, int site, double2& u0,
                                            double2 (&Un)[3], double2 (&W)[3],
                                            unsigned long long& rm) {
  u0 = L.u0[site];
#pragma unroll
  for (int j = 0; j < 3; ++j)
    Un[j] = FROM_U0 ? (XFORM ? make_double2(0.0, 0.0) : u0) : Uin.s[j][site];
  rm = 0ull;
  if (HAS_RBAR) {
    double2 r[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) r[m] = rb.s[m][site];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const double2 d = t_apply(j, r);
      Un[j].x += d.x;
      Un[j].y += d.y;
      rm = umax(rm, umax(abs_bits(d.x), abs_bits(d.y)));
    }
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double e0 = XFORM ? MB4_C[i] : MB4_E0[i];
    W[i].x = e0 * u0.x + MB4_E[i][0] * Un[0].x + MB4_E[i][1] * Un[1].x + MB4_E[i][2] * Un[2].x;
    W[i].y = e0 * u0.y + MB4_E[i][0] * Un[0].y + MB4_E[i][1] * Un[1].y + MB4_E[i][2] * Un[2].y;
  }
}

// Final update or residual pass of Newton iteration `fin.prev` (see top).
// `chk` skips the pass once an earlier iteration converged; `rslot` (may be
// NULL) receives ||(T (x) I) rbar||_inf, used by the kernel-level entry point.
template <bool FROM_U0, bool HAS_RBAR, bool XFORM>
__global__ __launch_bounds__(kTile) void k_update_residual(Lattice L, CPlanes3 Uin, Planes3 Uout,
                                                           CPlanes3 rb, Planes3 phib,
                                                           unsigned long long* rslot,
                                                           ConvCheck chk, ConvCheck fin,
                                                           double2* u0_out) {
  if (converged_at(chk)) return;
  __shared__ double2 sw[3][kTY + 2][kTX + 2];
  const int nx = L.nx, ny = L.ny;
  const TileCoord c = tile_coord(nx, ny);

  if (HAS_RBAR && converged_at(fin)) {
    // u_1 = U_{c_3} of the converged iterate, written over u_0 site by site.
    if (c.inside) {
      const int site = c.y * nx + c.x;
      double2 r[3];
#pragma unroll
      for (int m = 0; m < 3; ++m) r[m] = rb.s[m][site];
      double2 base = FROM_U0 ? L.u0[site] : Uin.s[2][site];
      if (XFORM && !FROM_U0) {
        const double2 u = L.u0[site];
        base = make_double2(u.x + base.x, u.y + base.y);
      }
      const double2 d = t_apply(2, r);
      u0_out[site] = make_double2(base.x + d.x, base.y + d.y);
    }
    return;
  }

  const int lx = threadIdx.x % kTX, ly = threadIdx.x / kTX;
  // Own position (wrapped when the tile overhangs the lattice: such a
  // position may still be the periodic neighbour of an inside site).
  const int gx = c.inside ? c.x : wrap(c.x, nx);
  const int gy = c.inside ? c.y : wrap(c.y, ny);
  const int site = gy * nx + gx;
  double2 u0, Un[3], W[3];
  unsigned long long rm;
  site_update<FROM_U0, HAS_RBAR, XFORM>(L, Uin, rb, site, u0, Un, W, rm);
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
    site_update<FROM_U0, HAS_RBAR, XFORM>(L, Uin, rb, hs, hu0, hUn, hW, hrm);
#pragma unroll
    for (int i = 0; i < 3; ++i) sw[i][hy][hx] = hW[i];
  }
  __syncthreads();

  if (c.inside) {
    const double t = L.t, g = site_g(L, site), h = L.h;
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
    // Cubic part (Eq. fIu2) by 6-node Gauss-Legendre, exact for degree 11
    // (XFORM: the nodes are u_0 + sum_j L_qj X_j, the l_j summing to one).
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const double l0 = XFORM ? 1.0 : MB4_GL_L[q][0];
      const double zp = l0 * u0.x + MB4_GL_L[q][1] * Un[0].x + MB4_GL_L[q][2] * Un[1].x +
                        MB4_GL_L[q][3] * Un[2].x;
      const double zq = l0 * u0.y + MB4_GL_L[q][1] * Un[0].y + MB4_GL_L[q][2] * Un[1].y +
                        MB4_GL_L[q][3] * Un[2].y;
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
      const double2 x = XFORM ? Un[i] : make_double2(Un[i].x - u0.x, Un[i].y - u0.y);
      phi[i].x = x.x - h * phi[i].x;
      phi[i].y = x.y - h * phi[i].y;
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
  if (rslot != nullptr) block_max_to<kTile>(rm, rslot);
}

// ---------------------------------------------------------------------------
// Per site, the 2x2 block I - h lambda_i J_site with J_site = [[a, bb],
// [-cc, -a]], a = 2 g p q, bb = A_jj + g (p^2 + 3 q^2), cc = A_jj +
// g (3 p^2 + q^2) (Eqs. JL, JR), is inverted exactly: its determinant is
// 1 + (h lambda)^2 (bb cc - a^2).  The hopping part of J couples neighbours
// through h lambda_i t (sum r_q, -sum r_p), taken from the previous iterate.
struct SiteBlock {
  double a, bb, cc;
};

__device__ __forceinline__ SiteBlock site_block(const Lattice& L, double2 u, double v, double g) {
  const double vs = v + L.shift;
  const double pp = u.x * u.x, qq = u.y * u.y;
  SiteBlock s;
  s.a = 2.0 * g * u.x * u.y;
  s.bb = vs + g * (pp + 3.0 * qq);
  s.cc = vs + g * (3.0 * pp + qq);
  return s;
}

// r = (I - hl J_site)^-1 b, given inv = 1 / det(I - hl J_site).  The inverse
// is inv * (I + hl J'), J' = [[a, bb], [-cc, -a]], applied as
// inv * (b + hl J' b): no product of hl with the site block is formed, so
// nothing per stage has to be kept across the sweeps.
__device__ __forceinline__ double2 block_solve(const SiteBlock& s, double hl, double inv, double bp,
                                               double bq) {
  const double jp = s.a * bp + s.bb * bq;
  const double jq = s.cc * bp + s.a * bq;
  return make_double2(inv * (bp + hl * jp), inv * (bq - hl * jq));
}

// Precision of the stage corrections and of the sweeps: RT = double, or
// float for the FP32 inner solves (everything else stays FP64).
template <class T>
struct Vec2;
template <>
struct Vec2<double> {
  using type = double2;
};
template <>
struct Vec2<float> {
  using type = float2;
};
template <class T>
using vec2_t = typename Vec2<T>::type;

__device__ __forceinline__ double2 to_d2(double2 v) { return v; }
__device__ __forceinline__ double2 to_d2(float2 v) { return make_double2(v.x, v.y); }

template <class T>
__device__ __forceinline__ vec2_t<T> vec2(T x, T y) {
  vec2_t<T> r;
  r.x = x;
  r.y = y;
  return r;
}

template <class T>
struct SiteBlockT {
  T a, bb, cc;
};

template <class T>
__device__ __forceinline__ SiteBlockT<T> block_in(const SiteBlock& s) {
  return SiteBlockT<T>{T(s.a), T(s.bb), T(s.cc)};
}

// As block_solve, in precision T.
template <class T>
__device__ __forceinline__ vec2_t<T> block_solve_t(const SiteBlockT<T>& s, T hl, T inv, T bp,
                                                   T bq) {
  const T jp = s.a * bp + s.bb * bq;
  const T jq = s.cc * bp + s.a * bq;
  return vec2<T>(inv * (bp + hl * jp), inv * (bq - hl * jq));
}

// 1 / det(I - h lambda_i J_site) for the three stages, d_i = 1 +
// (h lambda_i)^2 (bb cc - a^2).  In FP64 one division serves all three:
// inv_0 = d_1 d_2 / (d_0 d_1 d_2) and so on (a few ulp; the product of the
// d_i overflows only for potentials beyond 1e100).  FP32 divides per stage,
// where that product could overflow for large potentials.
template <class T>
__device__ __forceinline__ void block_invs(const SiteBlockT<T>& s, double h, T (&inv)[3]) {
  const T dd = s.bb * s.cc - s.a * s.a;
  T d[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const T hl = T(h * MB4_LAMBDA[i]);
    d[i] = T(1) + hl * hl * dd;
  }
  if (sizeof(T) == sizeof(double)) {
    const T d01 = d[0] * d[1];
    const T r = T(1) / (d01 * d[2]);
    const T t = d[2] * r;
    inv[0] = d[1] * t;
    inv[1] = d[0] * t;
    inv[2] = d01 * r;
  } else {
#pragma unroll
    for (int i = 0; i < 3; ++i) inv[i] = T(1) / d[i];
  }
}

// f(u_0) = S grad H = (A q + g n q, -(A p + g n p)) at one site, from u and
// its four neighbours a, b (x -/+ 1), d, e (y -/+ 1).
__device__ __forceinline__ double2 f_from(const Lattice& L, double2 u, double v, double g,
                                          double2 a, double2 b, double2 d, double2 e) {
  const double sp = (a.x + b.x) + (d.x + e.x);
  const double sq = (a.y + b.y) + (d.y + e.y);
  const double vs = v + L.shift;
  const double gn = g * (u.x * u.x + u.y * u.y);
  return make_double2(-L.t * sq + (vs + gn) * u.y, L.t * sp - (vs + gn) * u.x);
}

// All H + 1 block-Jacobi sweeps of one stage solve in one pass (temporal
// blocking).  A 512-thread block owns an output tile and loads the right-hand
// side, u_0 and V once on the tile plus an H-site halo; the first sweep (from
// r = 0) is local, the next H exchange neighbours through LDS, the valid zone
// shrinking by one ring per sweep, and only the tile's interior goes back to
// HBM.  Each region position computes the iterate of its (wrapped) lattice
// site from its own region neighbours, so lattices smaller than the region
// give the same values as large ones.  The region is RX x RY positions (32 x 32
// by default; Region lists the shapes built), two per thread, so the tile
// shrinks as the halo grows.
//
// Modes: kSolvePlain takes -Phibar from phib_in and writes rbar.  The others
// are Newton iteration 1: the right-hand side -Phibar_i = h TC_i f(u_0) is
// built in place (TC = T^-1 c) from u_0 staged in LDS on the region plus a
// one-site ring.  kSolveFirst writes rbar (with store_rhs the tile's Phibar
// too, for extra plain sweeps); kSolveFirstX writes X^1 = (T (x) I) rbar
// instead (the fused path), and kSolveFirstXPrev also applies the previous
// step's final update (PrevStep) to the u_0 it stages.  ||u_0||_inf goes to
// *u0max_slot if that is not NULL.
__host__ __device__ constexpr int region_x(int region) {
  return region == kRegion64x16 ? 64 : 32;
}
__host__ __device__ constexpr int region_y(int region) {
  return region == kRegion32x32 ? 32 : 16;
}

enum SolveMode : int { kSolvePlain = 0, kSolveFirst = 1, kSolveFirstX = 2, kSolveFirstXPrev = 3 };

struct FirstArgs {
  unsigned long long* u0max_slot;  // ||u_0||_inf target
  bool store_rhs;                  // also write Phibar of the tile
};

// Where member m's u_1 of this step goes (StepOut).
__device__ __forceinline__ double2* step_dst(const StepOut& so, const Multi& mu, int m) {
  return (mu.todo != nullptr && mu.step == mu.todo[m] - 1) ? so.home : so.next;
}

// Threads of a solve block: two region positions per thread, except for the
// 32 x 16 shape, which takes one.  Its blocks then run the shortest chain
// (78-80 VGPRs, six waves per SIMD), which pays on lattices too small to
// fill the chip with 32 x 32 blocks; on large lattices the tuner keeps the
// 32 x 32 shape.  The shapes give the same bits: multiply-adds are fused
// only within one source expression (-ffp-contract=on), whatever the
// unrolling.
constexpr int region_threads(int rx, int ry) { return rx == 32 && ry == 16 ? rx * ry : rx * ry / 2; }

// The work of one block of k_stage_solve on tile b of the lattice L (whose
// pointers, like every pointer here, are already moved to the block's
// member), in the LDS planes sr.  pmode (PREV): how this step's u_0 is
// formed (PrevStep): 0 as it is, 1 the previous step's u_0 + X_3, 2 the
// previous step's u_0 (it did not converge).  final_only (PREV): the member
// took its last step of the batch, and the tile gets only that step's final
// update.
template <int RX, int RY, int H, int MODE, class RT>
__device__ __forceinline__ void stage_solve_tile(const Lattice& L, CPlanes3 phib_in,
                                                 Planes3 phib_out, Planes3 out,
                                                 unsigned long long* rslot, FirstArgs fa,
                                                 const PrevStep& pv, int pmode, bool final_only,
                                                 int b, vec2_t<RT> (*sr)[RX * RY]) {
  constexpr bool FIRST = MODE != kSolvePlain;
  constexpr bool XOUT = MODE == kSolveFirstX || MODE == kSolveFirstXPrev;
  constexpr bool PREV = MODE == kSolveFirstXPrev;
  static_assert(XOUT || sizeof(RT) == sizeof(double), "FP32 solves exist on the fused path only");
  using R2 = vec2_t<RT>;
  constexpr int kSolveThreads = region_threads(RX, RY);
  const int tid = thread_index();
  constexpr int RN = RX * RY;
  constexpr int TSX = RX - 2 * H, TSY = RY - 2 * H;
  constexpr int PER = RN / kSolveThreads;
  static_assert(RN % kSolveThreads == 0, "region must be a whole number of passes");
  constexpr int UX = RX + 2, UN = FIRST ? UX * (RY + 2) : 1;
  // u_0 on the region plus a one-site ring (FIRST) shares the LDS of the
  // stage iterates: it is dead once the right-hand sides are formed.
  static_assert(UN * sizeof(double2) <= 3 * RN * sizeof(R2),
                "u_0 staging must fit the iterate buffer");
  double2* const su = reinterpret_cast<double2*>(&sr[0][0]);
  const int nx = L.nx, ny = L.ny;
  int tx0, ty0;
  strip_tile(b, (nx + TSX - 1) / TSX, (ny + TSY - 1) / TSY, tx0, ty0);
  tx0 *= TSX;
  ty0 *= TSY;
  const bool fast = nx >= RX + 2 && ny >= RY + 2;
  // This step's u_0 at one site when it comes from the previous step.
  auto u_prev = [&](int site) {
    double2 u = pv.u0[site];
    if (pmode == 1) {
      const double2 x = pv.X.s[2][site];
      u.x += x.x;
      u.y += x.y;
    }
    return u;
  };
  if (PREV && final_only) {
    if (pmode == 2 && pv.home == pv.u0) return;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int idx = tid + j * kSolveThreads;
      const int lx = idx % RX, ly = idx / RX;
      if (lx >= H && lx < H + TSX && ly >= H && ly < H + TSY && tx0 + lx - H < nx &&
          ty0 + ly - H < ny) {
        const int site = (ty0 + ly - H) * nx + (tx0 + lx - H);
        pv.home[site] = u_prev(site);
      }
    }
    return;
  }

  // Own positions first: their potential is loaded before the u_0 staging
  // below, so both sets of loads are in flight together.
  int gsite[PER];
  double vv[PER], gg[PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int idx = tid + j * kSolveThreads;
    const int lx = idx % RX, ly = idx / RX;
    gsite[j] = wrap_in(ty0 - H + ly, ny, fast) * nx + wrap_in(tx0 - H + lx, nx, fast);
    vv[j] = L.V[gsite[j]];
    gg[j] = site_g(L, gsite[j]);
  }
  if (FIRST) {
    // All loads of the staging first, then the stores, so that the rounds'
    // latencies overlap.
    constexpr int NS = (UN + kSolveThreads - 1) / kSolveThreads;
    double2 st[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      const int e = tid + k * kSolveThreads;
      if (e < UN) {
        const int ex = e % UX, ey = e / UX;
        const int site =
            wrap_in(ty0 - H - 1 + ey, ny, fast) * nx + wrap_in(tx0 - H - 1 + ex, nx, fast);
        st[k] = (PREV && pmode != 0) ? u_prev(site) : L.u0[site];
      }
    }
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      const int e = tid + k * kSolveThreads;
      if (e < UN) su[e] = st[k];
    }
    __syncthreads();
  }

  R2 rhs[PER][3];
  SiteBlockT<RT> blk[PER];
  RT inv[PER][3];
  NormAcc um;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int idx = tid + j * kSolveThreads;
    const int lx = idx % RX, ly = idx / RX;
    const int site = gsite[j];
    const int e = (ly + 1) * UX + lx + 1;
    const double2 u = FIRST ? su[e] : L.u0[site];
    const double v = vv[j];
    blk[j] = block_in<RT>(site_block(L, u, v, gg[j]));
    block_invs(blk[j], L.h, inv[j]);
    double2 f = make_double2(0.0, 0.0);
    if (FIRST) {
      f = f_from(L, u, v, gg[j], su[e - 1], su[e + 1], su[e - UX], su[e + UX]);
      const bool tile = lx >= H && lx < H + TSX && ly >= H && ly < H + TSY &&
                        tx0 + lx - H < nx && ty0 + ly - H < ny;
      if (tile) {
        um.add(u.x);
        um.add(u.y);
        if (PREV && pmode != 0) pv.next[site] = u;
      }
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      if (FIRST) {
        const double k = L.h * MB4_TC[i];
        rhs[j][i] = vec2<RT>(RT(k * f.x), RT(k * f.y));
      } else {
        const double2 ph = phib_in.s[i][site];
        rhs[j][i] = vec2<RT>(RT(-ph.x), RT(-ph.y));
      }
    }
  }
  if (FIRST) __syncthreads();  // every read of the u_0 staging is done
  // First sweep (from r = 0): the local 2x2 solves.
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int idx = tid + j * kSolveThreads;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const RT hl = RT(L.h * MB4_LAMBDA[i]);
      sr[i][idx] = block_solve_t(blk[j], hl, inv[j][i], rhs[j][i].x, rhs[j][i].y);
    }
  }
  // Sweeps 2 .. H+1, one stage at a time so that only one stage's new values
  // are live in registers.  One barrier per stage sweep: after it, the
  // previous stage's new values are stored (every read of that buffer is
  // done) and stage i is computed from LDS (its buffer was last stored before
  // at least one earlier barrier).
  R2 rn[PER];
#pragma unroll
  for (int s = 0; s < H; ++s) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const RT hl = RT(L.h * MB4_LAMBDA[i]);
      const RT ht = hl * RT(L.t);
      __syncthreads();
      if (s > 0 || i > 0) {
        const int ip = i == 0 ? 2 : i - 1;
#pragma unroll
        for (int j = 0; j < PER; ++j) {
          const int idx = tid + j * kSolveThreads;
          const int lx = idx % RX, ly = idx / RX;
          if (lx >= 1 && lx <= RX - 2 && ly >= 1 && ly <= RY - 2) sr[ip][idx] = rn[j];
        }
      }
#pragma unroll
      for (int j = 0; j < PER; ++j) {
        const int idx = tid + j * kSolveThreads;
        const int lx = idx % RX, ly = idx / RX;
        if (lx >= 1 && lx <= RX - 2 && ly >= 1 && ly <= RY - 2) {
          const R2 r1 = sr[i][idx - 1], r2 = sr[i][idx + 1];
          const R2 r3 = sr[i][idx - RX], r4 = sr[i][idx + RX];
          const RT sp = (r1.x + r2.x) + (r3.x + r4.x);
          const RT sq = (r1.y + r2.y) + (r3.y + r4.y);
          rn[j] = block_solve_t(blk[j], hl, inv[j][i], rhs[j][i].x - ht * sq,
                                rhs[j][i].y + ht * sp);
        }
      }
    }
  }
  if (H > 0) {
    __syncthreads();
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int idx = tid + j * kSolveThreads;
      const int lx = idx % RX, ly = idx / RX;
      if (lx >= 1 && lx <= RX - 2 && ly >= 1 && ly <= RY - 2) sr[2][idx] = rn[j];
    }
  }
  __syncthreads();
  // Interior (valid after all sweeps) back to HBM; positions of the tile that
  // overhang the lattice are not written.
  NormAcc rm;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int idx = tid + j * kSolveThreads;
    const int lx = idx % RX, ly = idx / RX;
    if (lx >= H && lx < H + TSX && ly >= H && ly < H + TSY && tx0 + lx - H < nx &&
        ty0 + ly - H < ny) {
      double2 r[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        r[i] = to_d2(sr[i][idx]);
        if (!XOUT) out.s[i][gsite[j]] = r[i];
        if (FIRST && fa.store_rhs)
          phib_out.s[i][gsite[j]] = make_double2(-double(rhs[j][i].x), -double(rhs[j][i].y));
      }
      if (XOUT || rslot != nullptr) {
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          const double2 d = t_apply(m, r);
          if (XOUT) out.s[m][gsite[j]] = d;
          rm.add(d.x);
          rm.add(d.y);
        }
      }
    }
  }
  if (rslot != nullptr) block_max_to<kSolveThreads>(rm.bits(), rslot);
  if (FIRST && fa.u0max_slot != nullptr) block_max_to<kSolveThreads>(um.bits(), fa.u0max_slot);
}

template <int RX, int RY, int H, int MODE, class RT>
__global__ __launch_bounds__(region_threads(RX, RY), sizeof(RT) == 4 ? 6 : 4) void k_stage_solve(
    Lattice L, CPlanes3 phib_in, Planes3 phib_out, Planes3 out, unsigned long long* rslot,
    ConvCheck chk, FirstArgs fa, Multi mu, PrevStep pv) {
  constexpr bool PREV = MODE == kSolveFirstXPrev;
  const Loc w = locate(mu, L, xcd_block(blockIdx.x, gridDim.x));
  int pmode = 0;
  if (PREV) {
    if (mu.todo != nullptr && mu.step - 1 >= mu.todo[w.m]) return;
    offset_check(pv.chk, w.rec);
    offset_check(pv.fin, w.rec);
    pmode = converged_at(pv.chk) ? 0 : (converged_at(pv.fin) ? 1 : 2);
    pv.u0 = offset_ptr(pv.u0, w.base);
    offset_planes(pv.X, w.base);
    pv.next = offset_ptr(pv.next, w.base);
    pv.home = offset_ptr(pv.home, w.base);
  }
  if (w.skip && pmode == 0) return;
  offset_check(chk, w.rec);
  if (converged_at(chk)) return;
  offset_planes(phib_in, w.base);
  offset_planes(phib_out, w.base);
  offset_planes(out, w.base);
  rslot = offset_ptr(rslot, w.rec);
  fa.u0max_slot = offset_ptr(fa.u0max_slot, w.rec);
  __shared__ vec2_t<RT> sr[3][RX * RY];
  stage_solve_tile<RX, RY, H, MODE, RT>(L, phib_in, phib_out, out, rslot, fa, pv, pmode,
                                        PREV && w.skip, w.b, sr);
}

// ---------------------------------------------------------------------------
// One Newton iteration's residual fused with the next iteration's stage solve,
// so that Phibar never goes through HBM.  The iterate is held as X^iter =
// U^iter - e (x) u_0 (StepOut).  For iteration `iter`:
//   Phibar^iter = (T^-1 (x) I) Phi(u_0 + X^iter)          (Eqs. Phidefinition, MB4_4)
//   rbar^{iter+1} = H + 1 block-Jacobi sweeps on (I - h lambda_i J) r = -Phibar^iter
//   X^{iter+1} = X^iter + (T (x) I) rbar^{iter+1}           (Eq. MB4_6)
//   rec[iter + 1] = ||(T (x) I) rbar^{iter+1}||_inf
// unless iteration iter already met the tolerance, in which case the block
// writes u_1 = u_0 + X^iter_3 for its tile (Sec. 2.2: c_3 = 1) and stops.
// With U_i = u_0 + X_i, the stage-i linear term is c_i u_0 + sum_j E_ij X_j
// (the E_ij with j = 0..3 sum to c_i), the quadrature nodes are z_q = u_0 +
// sum_j L_qj X_j (the l_j sum to one) and the residual is X_i - h (...).
// A block works on an RX x RY region (32 x 32 with 512 threads by default),
// region_threads() threads: W_i (Eq. fKu2) on the whole region in LDS, the
// residual on the region less one ring, the sweeps on shrinking rings, and
// the (RX - 2 - 2H) x (RY - 2 - 2H) tile in the middle is written back.  As
// in k_stage_solve, each region position computes the values of its (wrapped)
// lattice site from region neighbours only.  iterate_tile_body is the work of
// one block; k_iterate and k_member_run run it.

// X^iter of the tile is kept in LDS too when the stage planes and it fit
// this block's share of the CU's 160 KiB at the occupancy of the launch
// bounds (4 waves per SIMD); otherwise it is read again at the end.  Holding
// it in registers through the sweeps would spill.  iterate_park() is the
// number of its sites so kept (1 when it is read again).
constexpr int iterate_park(int rx, int ry, int h) {
  return (rx * ry * 48 + (rx - 2 - 2 * h) * (ry - 2 - 2 * h) * 48 + 64 <=
          160 * 1024 * (region_threads(rx, ry) / 64) / (4 * 4))
             ? (rx - 2 - 2 * h) * (ry - 2 - 2 * h)
             : 1;
}

// The work of one block of k_iterate on tile b of L (pointers moved to the
// block's member) in the LDS planes sb and the X park sx.  at: iteration
// iter - 1 already met the tolerance, and the tile gets u_1 = u_0 + X_3,
// written to dst.  stage3_only: of X^{iter+1} only X_3 is written.
template <int RX, int RY, int H, class RT>
__device__ __forceinline__ void iterate_tile_body(const Lattice& L, CPlanes3 Xin, Planes3 Xout,
                                                  unsigned long long* rnext, bool at,
                                                  double2* dst, bool stage3_only, int b,
                                                  double2 (*sb)[RX * RY],
                                                  double2 (*sx)[iterate_park(RX, RY, H)]) {
  using R2 = vec2_t<RT>;
  constexpr int kIterThreads = region_threads(RX, RY);
  const int tid = thread_index();
  constexpr int RN = RX * RY;
  constexpr int TSX = RX - 2 - 2 * H, TSY = RY - 2 - 2 * H;
  constexpr int PER = RN / kIterThreads;
  const int nx = L.nx, ny = L.ny;
  int tx0, ty0;
  strip_tile(b, (nx + TSX - 1) / TSX, (ny + TSY - 1) / TSY, tx0, ty0);
  tx0 *= TSX;
  ty0 *= TSY;
  const int ox = tx0 - H - 1, oy = ty0 - H - 1;  // region origin
  const bool fast = nx >= RX + 2 && ny >= RY + 2;

  if (at) {
    // Final update on this block's tile only.
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int idx = tid + j * kIterThreads;
      const int lx = idx % RX, ly = idx / RX;
      if (lx >= H + 1 && lx < H + 1 + TSX && ly >= H + 1 && ly < H + 1 + TSY &&
          ox + lx < nx && oy + ly < ny) {
        const int site = (oy + ly) * nx + (ox + lx);
        const double2 u = L.u0[site], x = Xin.s[2][site];
        dst[site] = make_double2(u.x + x.x, u.y + x.y);
      }
    }
    return;
  }

  // W_i (FP64), then the stage iterates (RT) in the same LDS, and X^iter
  // of the tile parked in sx (iterate_park).
  constexpr bool XLDS = iterate_park(RX, RY, H) > 1;
  R2(*const si)[RN] = reinterpret_cast<R2(*)[RN]>(&sb[0][0]);
  int gsite[PER];
  double2 u0v[PER];
  double2 xv[PER][3];
  double vv[PER], gg[PER];
  // Phase 1: W_i on the whole region.  Every load of both positions is
  // issued before the first LDS store, so that their latencies overlap.
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int idx = tid + j * kIterThreads;
    const int lx = idx % RX, ly = idx / RX;
    const int site = wrap_in(oy + ly, ny, fast) * nx + wrap_in(ox + lx, nx, fast);
    gsite[j] = site;
    u0v[j] = L.u0[site];
    vv[j] = L.V[site];
    gg[j] = site_g(L, site);
#pragma unroll
    for (int i = 0; i < 3; ++i) xv[j][i] = Xin.s[i][site];
  }
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int idx = tid + j * kIterThreads;
    if (XLDS) {
      const int tx = idx % RX - (H + 1), ty = idx / RX - (H + 1);
      if (tx >= 0 && tx < TSX && ty >= 0 && ty < TSY) {
#pragma unroll
        for (int i = 0; i < 3; ++i) sx[i][ty * TSX + tx] = xv[j][i];
      }
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      sb[i][idx] = make_double2(MB4_C[i] * u0v[j].x + MB4_E[i][0] * xv[j][0].x +
                                    MB4_E[i][1] * xv[j][1].x + MB4_E[i][2] * xv[j][2].x,
                                MB4_C[i] * u0v[j].y + MB4_E[i][0] * xv[j][0].y +
                                    MB4_E[i][1] * xv[j][1].y + MB4_E[i][2] * xv[j][2].y);
    }
  }
  __syncthreads();

  // Phase 2: residual and transform on ring >= 1.
  R2 rhs[PER][3];
  SiteBlockT<RT> blk[PER];
  RT inv[PER][3];
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int idx = tid + j * kIterThreads;
    const int lx = idx % RX, ly = idx / RX;
    blk[j] = block_in<RT>(site_block(L, u0v[j], vv[j], gg[j]));
    if (lx >= 1 && lx <= RX - 2 && ly >= 1 && ly <= RY - 2) {
      block_invs(blk[j], L.h, inv[j]);
      const double t = L.t, g = gg[j], h = L.h;
      const double vs = vv[j] + L.shift;
      double2 phi[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const double2 w = sb[i][idx];
        const double2 l = sb[i][idx - 1], r = sb[i][idx + 1];
        const double2 d = sb[i][idx - RX], u = sb[i][idx + RX];
        const double sp = (l.x + r.x) + (d.x + u.x);
        const double sq = (l.y + r.y) + (d.y + u.y);
        phi[i] = make_double2(-t * sq + vs * w.y, t * sp - vs * w.x);
      }
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        const double zp = u0v[j].x + MB4_GL_L[q][1] * xv[j][0].x +
                          MB4_GL_L[q][2] * xv[j][1].x + MB4_GL_L[q][3] * xv[j][2].x;
        const double zq = u0v[j].y + MB4_GL_L[q][1] * xv[j][0].y +
                          MB4_GL_L[q][2] * xv[j][1].y + MB4_GL_L[q][3] * xv[j][2].y;
        const double gn = g * (zp * zp + zq * zq);
        const double fp = gn * zq, fq = -gn * zp;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          phi[i].x += MB4_GL_Q[i][q] * fp;
          phi[i].y += MB4_GL_Q[i][q] * fq;
        }
      }
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        phi[i].x = xv[j][i].x - h * phi[i].x;
        phi[i].y = xv[j][i].y - h * phi[i].y;
      }
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const double bp = MB4_TINV[i][0] * phi[0].x + MB4_TINV[i][1] * phi[1].x +
                          MB4_TINV[i][2] * phi[2].x;
        const double bq = MB4_TINV[i][0] * phi[0].y + MB4_TINV[i][1] * phi[1].y +
                          MB4_TINV[i][2] * phi[2].y;
        rhs[j][i] = vec2<RT>(RT(-bp), RT(-bq));
      }
    }
  }
  __syncthreads();  // every stencil read of W is done
  // First sweep (from r = 0, local) on ring >= 1, formed only now so that
  // its values need no registers across the barrier.
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int idx = tid + j * kIterThreads;
    const int lx = idx % RX, ly = idx / RX;
    if (lx >= 1 && lx <= RX - 2 && ly >= 1 && ly <= RY - 2) {
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const RT hl = RT(L.h * MB4_LAMBDA[i]);
        si[i][idx] = block_solve_t(blk[j], hl, inv[j][i], rhs[j][i].x, rhs[j][i].y);
      }
    }
  }
  // Sweeps 2 .. H+1 on ring >= 2, one stage at a time with one barrier per
  // stage sweep (see k_stage_solve).
  R2 rn[PER];
#pragma unroll
  for (int s = 0; s < H; ++s) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const RT hl = RT(L.h * MB4_LAMBDA[i]);
      const RT ht = hl * RT(L.t);
      __syncthreads();
      if (s > 0 || i > 0) {
        const int ip = i == 0 ? 2 : i - 1;
#pragma unroll
        for (int j = 0; j < PER; ++j) {
          const int idx = tid + j * kIterThreads;
          const int lx = idx % RX, ly = idx / RX;
          if (lx >= 2 && lx <= RX - 3 && ly >= 2 && ly <= RY - 3) si[ip][idx] = rn[j];
        }
      }
#pragma unroll
      for (int j = 0; j < PER; ++j) {
        const int idx = tid + j * kIterThreads;
        const int lx = idx % RX, ly = idx / RX;
        if (lx >= 2 && lx <= RX - 3 && ly >= 2 && ly <= RY - 3) {
          const R2 q1 = si[i][idx - 1], q2 = si[i][idx + 1];
          const R2 q3 = si[i][idx - RX], q4 = si[i][idx + RX];
          const RT sp = (q1.x + q2.x) + (q3.x + q4.x);
          const RT sq = (q1.y + q2.y) + (q3.y + q4.y);
          rn[j] = block_solve_t(blk[j], hl, inv[j][i], rhs[j][i].x - ht * sq,
                                rhs[j][i].y + ht * sp);
        }
      }
    }
  }
  // Tile positions never wrap, so their site is formed afresh here (reusing
  // the phase-1 addresses would keep them live, and spilled, all along).
  int tsite[PER];
  double2 xt[PER][3];
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int idx = tid + j * kIterThreads;
    const int lx = idx % RX, ly = idx / RX;
    const bool tile = lx >= H + 1 && lx < H + 1 + TSX && ly >= H + 1 && ly < H + 1 + TSY &&
                      ox + lx < nx && oy + ly < ny;
    tsite[j] = tile ? (oy + ly) * nx + (ox + lx) : -1;
    if (tile && !XLDS) {
#pragma unroll
      for (int m = 0; m < 3; ++m) xt[j][m] = Xin.s[m][tsite[j]];
    }
  }
  if (H > 0) {
    __syncthreads();
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int idx = tid + j * kIterThreads;
      const int lx = idx % RX, ly = idx / RX;
      if (lx >= 2 && lx <= RX - 3 && ly >= 2 && ly <= RY - 3) si[2][idx] = rn[j];
    }
  }
  __syncthreads();
  // The tile: X^{iter+1} back to HBM, and the update norm.
  NormAcc rm;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int idx = tid + j * kIterThreads;
    if (tsite[j] >= 0) {
      if (XLDS) {
        const int tp = (idx / RX - (H + 1)) * TSX + (idx % RX - (H + 1));
#pragma unroll
        for (int m = 0; m < 3; ++m) xt[j][m] = sx[m][tp];
      }
      double2 r[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) r[i] = to_d2(si[i][idx]);
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        const double2 d = t_apply(m, r);
        if (!stage3_only || m == 2)
          Xout.s[m][tsite[j]] = make_double2(xt[j][m].x + d.x, xt[j][m].y + d.y);
        rm.add(d.x);
        rm.add(d.y);
      }
    }
  }
  block_max_to<kIterThreads>(rm.bits(), rnext);
}

template <int RX, int RY, int H, class RT>
__global__ __launch_bounds__(region_threads(RX, RY), 4) void k_iterate(Lattice L, CPlanes3 Xin, Planes3 Xout,
                                                          unsigned long long* rnext,
                                                          ConvCheck chk, ConvCheck fin,
                                                          StepOut so, Multi mu) {
  const Loc w = locate(mu, L, xcd_block(blockIdx.x, gridDim.x));
  if (w.skip) return;
  offset_check(chk, w.rec);
  offset_check(fin, w.rec);
  rnext = offset_ptr(rnext, w.rec);
  if (converged_at(chk)) return;
  const bool at = converged_at(fin);
  offset_planes(Xin, w.base);
  offset_planes(Xout, w.base);
  double2* const dst = at ? offset_ptr(step_dst(so, mu, w.m), w.base) : nullptr;
  __shared__ double2 sb[3][RX * RY];
  __shared__ double2 sx[3][iterate_park(RX, RY, H)];
  iterate_tile_body<RX, RY, H, RT>(L, Xin, Xout, rnext, at, dst, so.stage3_only, w.b, sb, sx);
}

// Final update of the last step of a batch, site by site (launch_final_update).
__global__ __launch_bounds__(kFinalSites) void k_final_update(Lattice L, CPlanes3 X,
                                                              ConvCheck chk, ConvCheck fin,
                                                              StepOut so, int n, Multi mu) {
  const Loc w = locate(mu, L, xcd_block(blockIdx.x, gridDim.x));
  if (w.skip) return;
  offset_check(chk, w.rec);
  offset_check(fin, w.rec);
  if (converged_at(chk)) return;
  const bool at = converged_at(fin);
  double2* const dst = offset_ptr(step_dst(so, mu, w.m), w.base);
  if (!at && dst == L.u0) return;
  if (mu.desc != nullptr) n = L.nx * L.ny;
  offset_planes(X, w.base);
  const int site = w.b * kFinalSites + threadIdx.x;
  if (site >= n) return;
  double2 u = L.u0[site];
  if (at) {
    const double2 x = X.s[2][site];
    u.x += x.x;
    u.y += x.y;
  }
  dst[site] = u;
}

// A value every lane of the wave holds, moved to scalar registers.
__device__ __forceinline__ double uniform_double(double x) {
  const long long b = __double_as_longlong(x);
  const unsigned lo = static_cast<unsigned>(__builtin_amdgcn_readfirstlane(static_cast<int>(b)));
  const long long hi = __builtin_amdgcn_readfirstlane(static_cast<int>(b >> 32));
  return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

__device__ __forceinline__ MemberDesc uniform_desc(const MemberDesc& d) {
  MemberDesc u;
  u.nx = __builtin_amdgcn_readfirstlane(d.nx);
  u.ny = __builtin_amdgcn_readfirstlane(d.ny);
  u.t = uniform_double(d.t);
  u.shift = uniform_double(d.shift);
  u.g = uniform_double(d.g);
  u.h = uniform_double(d.h);
  const unsigned lo = static_cast<unsigned>(__builtin_amdgcn_readfirstlane(static_cast<int>(d.base)));
  const long long hi = __builtin_amdgcn_readfirstlane(static_cast<int>(d.base >> 32));
  u.base = static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo);
  return u;
}

// A batch of the multi-lattice engine in one launch (MemberRun): block w
// takes its members one after the other through all their steps.  Each
// Newton iteration of a step is the member's tiles, walked in the order of
// the per-phase launches, with the same tile bodies and the same LDS layout,
// so the results are those of the per-phase launches bit for bit.  The
// update norm of the iteration in progress is reduced into LDS (rec[1];
// ||u_0||_inf in rec[0]), and thread 0 alone takes the decision, which the
// block reads after a barrier: every thread follows the same branch.
template <int RX, int RY, int H, class RT>
__global__ __launch_bounds__(region_threads(RX, RY), 4) void k_member_run(Lattice base,
                                                                          MemberRun run) {
  using R2 = vec2_t<RT>;
  constexpr int NT = region_threads(RX, RY);
  constexpr int RN = RX * RY;
  constexpr int PARK = iterate_park(RX, RY, H);
  constexpr size_t kSolveBytes = sizeof(R2) * 3 * RN;
  constexpr size_t kIterBytes = sizeof(double2) * 3 * (RN + PARK);
  __shared__ __align__(16) unsigned char arena[kSolveBytes > kIterBytes ? kSolveBytes : kIterBytes];
  __shared__ unsigned long long rec[2];
  __shared__ int verdict;
  R2(*const sr)[RN] = reinterpret_cast<R2(*)[RN]>(arena);
  double2(*const sb)[RN] = reinterpret_cast<double2(*)[RN]>(arena);
  double2(*const sx)[PARK] = reinterpret_cast<double2(*)[PARK]>(arena + sizeof(double2) * 3 * RN);
  constexpr int FSX = RX - 2 * H, FSY = RY - 2 * H;          // tile of the first solve
  constexpr int ISX = RX - 2 - 2 * H, ISY = RY - 2 - 2 * H;  // tile of an iteration
  const CPlanes3 cnone{{nullptr, nullptr, nullptr}};
  const Planes3 none{{nullptr, nullptr, nullptr}};
  // Thread 0's verdict on the iteration just done: 1 converged, 0 not yet,
  // -1 a norm that is not finite.
  auto decide = [&]() {
    __syncthreads();
    if (threadIdx.x == 0) {
      const double r = bits_double(rec[1]);
      const double tol = run.relative ? conv_tol(run.eps, bits_double(rec[0])) : run.eps;
      verdict = r <= tol ? 1 : (isfinite(r) ? 0 : -1);
      rec[1] = 0ull;
    }
    __syncthreads();
    return verdict;
  };
  for (int k = run.wfirst[blockIdx.x]; k < run.wfirst[blockIdx.x + 1]; ++k) {
    // The member and its descriptor are the same for the whole block; read
    // through the first lane, they stay in scalar registers.
    const int m = __builtin_amdgcn_readfirstlane(run.order[k]);
    const MemberDesc d = uniform_desc(run.desc[m]);
    Lattice L = base;
    L.nx = d.nx;
    L.ny = d.ny;
    L.t = d.t;
    L.shift = d.shift;
    L.g = d.g;
    L.h = d.h;
    L.V += d.base;
    if (L.gs != nullptr) L.gs += d.base;
    const int nf = ((d.nx + FSX - 1) / FSX) * ((d.ny + FSY - 1) / FSY);
    const int ni = ((d.nx + ISX - 1) / ISX) * ((d.ny + ISY - 1) / ISY);
    double2* const home = run.u0 + d.base;
    auto u0_of = [&](int step) { return ((step & 1) ? run.u0b : run.u0) + d.base; };
    auto x_of = [&](int par) {
      double2* const* a = par ? run.Xa : run.Xb;
      return Planes3{{a[0] + d.base, a[1] + d.base, a[2] + d.base}};
    };
    auto cx_of = [&](int par) {
      const Planes3 p = x_of(par);
      return CPlanes3{{p.s[0], p.s[1], p.s[2]}};
    };
    int par = 0;  // X^l of the step in progress lives in x_of(par)
    const int steps = run.todo[m];
    // Predicted iteration count: its iteration writes only X_3 (as the
    // per-phase form's last iteration does); a step that needs more is taken
    // again from its u_0 with one iteration more.  It follows a count up at
    // once and down after two lower steps.
    int pred = __builtin_amdgcn_readfirstlane(run.pred[m]), lower = 0;
    for (int step = 0; step < steps; ++step) {
      if (threadIdx.x == 0) rec[0] = rec[1] = 0ull;
      __syncthreads();
      const FirstArgs fa{run.relative ? &rec[0] : nullptr, false};
      const ConvCheck nochk{nullptr, 0, 0.0, false};
      const PrevStep pv{u0_of(step - 1), cx_of(par), nochk, nochk, u0_of(step), home};
      L.u0 = u0_of(step);
      // pmode 1: this step's u_0 is formed from the previous step's by the
      // first solve (and written to u0_of(step)); 0 on the member's first
      // step of the batch and when a step is taken again.
      int pmode = step > 0 ? 1 : 0;
      int it, v;
      for (;;) {
        // Newton iteration 1, fused with the previous step's final update.
        for (int b = 0; b < nf; ++b)
          stage_solve_tile<RX, RY, H, kSolveFirstXPrev, RT>(L, cnone, none, x_of(par ^ 1),
                                                            &rec[1], fa, pv, pmode, false, b, sr);
        par ^= 1;
        it = 1;
        v = decide();
        bool short_of = false;
        while (v == 0 && it < run.max_newton) {
          const bool last = it + 1 == pred;
          for (int b = 0; b < ni; ++b)
            iterate_tile_body<RX, RY, H, RT>(L, cx_of(par), x_of(par ^ 1), &rec[1], false,
                                             nullptr, last, b, sb, sx);
          par ^= 1;
          ++it;
          v = decide();
          if (v == 0 && last && it < run.max_newton) {
            short_of = true;
            break;
          }
        }
        if (!short_of) break;
        pred = it + 1;
        lower = 0;
        pmode = 0;
      }
      if (v == 1) {
        if (it >= pred) {
          pred = it;
          lower = 0;
        } else if (++lower >= 2) {
          pred = it;
          lower = 0;
        }
      }
      if (threadIdx.x == 0) run.conv[step * run.members + m] = v == 1 ? it : (v < 0 ? -1 : 0);
      if (v != 1) {
        // The step failed for good: the member keeps this step's u_0.
        if (step & 1) {
          const double2* const src = u0_of(step);
          for (int i = threadIdx.x; i < d.nx * d.ny; i += NT) home[i] = src[i];
        }
        break;
      }
      if (step == steps - 1) {
        // u_1 = u_0 + X_3 of the converged iterate, into the home buffer,
        // site by site (home may be this step's u_0).
        const double2* const u = L.u0;
        const double2* const x3 = x_of(par).s[2];
        for (int i = thread_index(); i < d.nx * d.ny; i += NT) {
          const double2 a = u[i], x = x3[i];
          home[i] = make_double2(a.x + x.x, a.y + x.y);
        }
      }
    }
    if (threadIdx.x == 0) run.pred[m] = pred;
    __syncthreads();
  }
}

// One more block-Jacobi sweep from the iterate rin (solves with more than
// four sweeps); rslot (may be NULL) receives ||(T (x) I) rout||_inf.
__global__ __launch_bounds__(kTile) void k_stage_sweep(Lattice L, CPlanes3 phib, CPlanes3 rin,
                                                       Planes3 rout, unsigned long long* rslot,
                                                       ConvCheck chk) {
  if (converged_at(chk)) return;
  const int nx = L.nx, ny = L.ny;
  const TileCoord c = tile_coord(nx, ny);
  unsigned long long rm = 0ull;
  if (c.inside) {
    const int site = c.y * nx + c.x;
    const SiteBlock blk = site_block(L, L.u0[site], L.V[site], site_g(L, site));
    const int xl = c.x == 0 ? nx - 1 : c.x - 1, xr = c.x == nx - 1 ? 0 : c.x + 1;
    const int yd = c.y == 0 ? ny - 1 : c.y - 1, yu = c.y == ny - 1 ? 0 : c.y + 1;
    const int sl = c.y * nx + xl, sr = c.y * nx + xr, sd = yd * nx + c.x, su = yu * nx + c.x;
    double2 r[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double hl = L.h * MB4_LAMBDA[i];
      const double2 ph = phib.s[i][site];
      const double2 r1 = rin.s[i][sl], r2 = rin.s[i][sr], r3 = rin.s[i][sd], r4 = rin.s[i][su];
      const double sp = (r1.x + r2.x) + (r3.x + r4.x);
      const double sq = (r1.y + r2.y) + (r3.y + r4.y);
      const double ht = hl * L.t;
      const double inv = 1.0 / (1.0 + hl * hl * (blk.bb * blk.cc - blk.a * blk.a));
      r[i] = block_solve(blk, hl, inv, -ph.x - ht * sq, -ph.y + ht * sp);
      rout.s[i][site] = r[i];
    }
    if (rslot != nullptr) {
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        const double2 d = t_apply(m, r);
        rm = umax(rm, umax(abs_bits(d.x), abs_bits(d.y)));
      }
    }
  }
  if (rslot != nullptr) block_max_to<kTile>(rm, rslot);
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

// Error-free product: a * b = hi + lo exactly (one FMA).
__device__ __forceinline__ DD two_prod(double a, double b) {
  const double p = a * b;
  return DD{p, fma(a, b, -p)};
}

// Error-free sum (Knuth): a + b = hi + lo exactly.
__device__ __forceinline__ DD two_sum(double a, double b) {
  const double s = a + b;
  const double bb = s - a;
  return DD{s, (a - (s - bb)) + (b - bb)};
}

// x * c and x * y to about twice the working precision.
__device__ __forceinline__ DD dd_mul(DD x, double c) {
  const DD p = two_prod(x.hi, c);
  const double e = p.lo + x.lo * c;
  const double hi = p.hi + e;
  return DD{hi, e - (hi - p.hi)};
}

__device__ __forceinline__ DD dd_mul(DD x, DD y) {
  const DD p = two_prod(x.hi, y.hi);
  const double e = p.lo + (x.hi * y.lo + x.lo * y.hi);
  const double hi = p.hi + e;
  return DD{hi, e - (hi - p.hi)};
}

// x * 2^k (exact).
__device__ __forceinline__ DD dd_scale(DD x, double pow2) { return DD{x.hi * pow2, x.lo * pow2}; }

constexpr int kEnergyParts = 6;

// psi at a site: from the interleaved L.u0, or (kPlanes) from two planes p, q
// of nx*ny doubles each.
struct PsiPlanes {
  const double* p;
  const double* q;
};

template <bool kPlanes>
__device__ __forceinline__ double2 psi_at(const Lattice& L, const PsiPlanes& pl, int site) {
  if constexpr (kPlanes)
    return make_double2(pl.p[site], pl.q[site]);
  else
    return L.u0[site];
}

// Per-block sums of the six energy terms; partials[(block*6 + k)*2 + {0,1}]
// with block the XCD-remapped index, so that a member's blocks are
// contiguous.
template <bool kPlanes>
__global__ __launch_bounds__(kTile) void k_energy_partial(Lattice L, double* partials, Multi mu,
                                                          PsiPlanes pl) {
  __shared__ DD red[kEnergyParts][kTile];
  const int bl = xcd_block(blockIdx.x, gridDim.x);
  const Loc w = locate(mu, L, bl);
  const int nx = L.nx, ny = L.ny;
  const TileCoord c = tile_coord_at(nx, ny, w.b);
  DD v[kEnergyParts];
#pragma unroll
  for (int k = 0; k < kEnergyParts; ++k) v[k] = DD{0.0, 0.0};
  if (c.inside) {
    // Each site's terms are formed in double-double from the exact inputs,
    // so no rounding is left at the size of the terms themselves.  That
    // matters where they cancel: with a diagonal shift 4t (the continuum
    // -Delta_h), shift * n and t * (u . sum of neighbours) are both about
    // 4 t n for a smooth field, and their difference, the kinetic energy
    // density, is far smaller.
    const int site = c.y * nx + c.x;
    const int xl = c.x == 0 ? nx - 1 : c.x - 1, xr = c.x == nx - 1 ? 0 : c.x + 1;
    const int yd = c.y == 0 ? ny - 1 : c.y - 1, yu = c.y == ny - 1 ? 0 : c.y + 1;
    const double2 u = psi_at<kPlanes>(L, pl, site);
    const double2 a = psi_at<kPlanes>(L, pl, c.y * nx + xl);
    const double2 b = psi_at<kPlanes>(L, pl, c.y * nx + xr);
    const double2 d = psi_at<kPlanes>(L, pl, yd * nx + c.x);
    const double2 e = psi_at<kPlanes>(L, pl, yu * nx + c.x);
    const DD sp = dd_add(two_sum(a.x, b.x), two_sum(d.x, e.x));
    const DD sq = dd_add(two_sum(a.y, b.y), two_sum(d.y, e.y));
    const DD n = dd_add(two_prod(u.x, u.x), two_prod(u.y, u.y));
    const DD hop = dd_add(dd_mul(sp, u.x), dd_mul(sq, u.y));
    const DD uk = dd_scale(dd_add(dd_mul(n, L.shift), dd_mul(hop, -L.t)), 0.5);
    const DD ue = dd_scale(dd_mul(n, L.V[site]), 0.5);
    const DD n2 = dd_mul(n, n);
    const DD ui = dd_scale(dd_mul(n2, site_g(L, site)), 0.25);
    v[0] = dd_add(dd_add(uk, ue), ui);
    v[1] = uk;
    v[2] = ui;
    v[3] = ue;
    v[4] = n;
    v[5] = n2;
  }
#pragma unroll
  for (int k = 0; k < kEnergyParts; ++k) red[k][threadIdx.x] = v[k];
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
    partials[(static_cast<size_t>(bl) * kEnergyParts + threadIdx.x) * 2 + 0] = s.hi;
    partials[(static_cast<size_t>(bl) * kEnergyParts + threadIdx.x) * 2 + 1] = s.lo;
  }
}

// Sum of the partials of blocks [first, last) into out[0 .. 6), in a fixed
// order.  One block per output: block m of a Multi sums member m's blocks.
__global__ __launch_bounds__(kTile) void k_energy_final(const double* partials, int nblocks,
                                                         const int* block0, double* out) {
  __shared__ DD red[kEnergyParts][kTile];
  int first = 0, last = nblocks;
  if (block0 != nullptr) {
    first = block0[blockIdx.x];
    last = block0[blockIdx.x + 1];
    out += kEnergyParts * blockIdx.x;
  }
  DD acc[kEnergyParts];
#pragma unroll
  for (int k = 0; k < kEnergyParts; ++k) acc[k] = DD{0.0, 0.0};
  for (int bkt = first + threadIdx.x; bkt < last; bkt += kTile) {
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
// A timed launch goes through hipExtLaunchKernelGGL, so that the start/stop
// timestamps are taken by the dispatch itself (no extra marker packets
// between kernels); an untimed one is a plain launch (which stream capture
// into graphs records as a kernel node).
#define MB4_LAUNCH(kernel, grid, block, ev, ...)                                             \
  do {                                                                                       \
    if ((ev).start == nullptr && (ev).stop == nullptr)                                       \
      hipLaunchKernelGGL(kernel, grid, block, 0, stream, __VA_ARGS__);                       \
    else                                                                                     \
      hipExtLaunchKernelGGL(kernel, grid, block, 0, stream, (ev).start, (ev).stop, 0u,      \
                            __VA_ARGS__);                                                    \
    return hipGetLastError();                                                                \
  } while (0)

hipError_t launch_clear(unsigned long long* p, int n, hipStream_t stream) {
  const int blocks = std::max(1, std::min((n + 255) / 256, 64));
  MB4_LAUNCH(k_clear_u64, dim3(blocks), dim3(256), LaunchEvents{}, p, n);
}

hipError_t launch_member_table(const int* block0, int count, int blocks, int* member_of,
                               hipStream_t stream) {
  if (blocks <= 0) return hipSuccess;
  MB4_LAUNCH(k_member_table, dim3((blocks + 255) / 256), dim3(256), LaunchEvents{}, block0, count,
             blocks, member_of);
}

hipError_t launch_update_residual(const Lattice& lat, CPlanes3 Uin, Planes3 Uout, CPlanes3 rbar,
                                  bool has_rbar, bool from_u0, Planes3 phib,
                                  unsigned long long* rslot, ConvCheck check, ConvCheck fin,
                                  double2* u0_out, hipStream_t stream, LaunchEvents ev,
                                  bool xform) {
  const dim3 grid(tile_blocks(lat.nx, lat.ny)), block(kTile);
#define MB4_UPD(F, R, X)                                                                      \
  MB4_LAUNCH((k_update_residual<F, R, X>), grid, block, ev, lat, Uin, Uout, rbar, phib, rslot, \
             check, fin, u0_out)
  if (xform) {
    if (from_u0 && has_rbar) MB4_UPD(true, true, true);
    if (from_u0) MB4_UPD(true, false, true);
    if (has_rbar) MB4_UPD(false, true, true);
    MB4_UPD(false, false, true);
  }
  if (from_u0 && has_rbar) MB4_UPD(true, true, false);
  if (from_u0) MB4_UPD(true, false, false);
  if (has_rbar) MB4_UPD(false, true, false);
  MB4_UPD(false, false, false);
#undef MB4_UPD
}

const char* region_name(int region) {
  switch (region) {
    case kRegion32x32: return "32x32";
    case kRegion64x16: return "64x16";
    case kRegion32x16: return "32x16";
    default: return "?";
  }
}

void first_solve_tile(int region, int sweeps, int* tx, int* ty) {
  *tx = region_x(region) - 2 * (sweeps - 1);
  *ty = region_y(region) - 2 * (sweeps - 1);
}

void iterate_tile(int region, int sweeps, int* tx, int* ty) {
  *tx = region_x(region) - 2 - 2 * (sweeps - 1);
  *ty = region_y(region) - 2 - 2 * (sweeps - 1);
}

void energy_tile(int* tx, int* ty) {
  *tx = kTX;
  *ty = kTY;
}

namespace {

template <int RX, int RY, int MODE, class RT>
hipError_t launch_solve_region(const Lattice& lat, CPlanes3 phib_in, Planes3 phib_out,
                               Planes3 out, unsigned long long* rslot, ConvCheck check,
                               FirstArgs fa, int sweeps, const Multi& mu, hipStream_t stream,
                               LaunchEvents ev, PrevStep pv = PrevStep{}) {
  const int h = sweeps - 1, tx = RX - 2 * h, ty = RY - 2 * h;
  const dim3 grid(mu.desc != nullptr ? mu.blocks
                                     : ((lat.nx + tx - 1) / tx) * ((lat.ny + ty - 1) / ty)),
      block(region_threads(RX, RY));
  switch (sweeps) {
    case 1:
      MB4_LAUNCH((k_stage_solve<RX, RY, 0, MODE, RT>), grid, block, ev, lat, phib_in, phib_out,
                 out, rslot, check, fa, mu, pv);
    case 2:
      MB4_LAUNCH((k_stage_solve<RX, RY, 1, MODE, RT>), grid, block, ev, lat, phib_in, phib_out,
                 out, rslot, check, fa, mu, pv);
    case 3:
      MB4_LAUNCH((k_stage_solve<RX, RY, 2, MODE, RT>), grid, block, ev, lat, phib_in, phib_out,
                 out, rslot, check, fa, mu, pv);
    case 4:
      MB4_LAUNCH((k_stage_solve<RX, RY, 3, MODE, RT>), grid, block, ev, lat, phib_in, phib_out,
                 out, rslot, check, fa, mu, pv);
    default:
      return hipErrorInvalidValue;
  }
}

template <int RX, int RY, class RT>
hipError_t launch_iterate_region(const Lattice& lat, CPlanes3 Xin, Planes3 Xout, int sweeps,
                                 unsigned long long* rnext, ConvCheck check, ConvCheck fin,
                                 StepOut so, const Multi& mu, hipStream_t stream,
                                 LaunchEvents ev) {
  const int h = sweeps - 1, tx = RX - 2 - 2 * h, ty = RY - 2 - 2 * h;
  const dim3 grid(mu.desc != nullptr ? mu.blocks
                                     : ((lat.nx + tx - 1) / tx) * ((lat.ny + ty - 1) / ty)),
      block(region_threads(RX, RY));
  switch (sweeps) {
    case 1:
      MB4_LAUNCH((k_iterate<RX, RY, 0, RT>), grid, block, ev, lat, Xin, Xout, rnext, check, fin,
                 so, mu);
    case 2:
      MB4_LAUNCH((k_iterate<RX, RY, 1, RT>), grid, block, ev, lat, Xin, Xout, rnext, check, fin,
                 so, mu);
    case 3:
      MB4_LAUNCH((k_iterate<RX, RY, 2, RT>), grid, block, ev, lat, Xin, Xout, rnext, check, fin,
                 so, mu);
    case 4:
      MB4_LAUNCH((k_iterate<RX, RY, 3, RT>), grid, block, ev, lat, Xin, Xout, rnext, check, fin,
                 so, mu);
    default:
      return hipErrorInvalidValue;
  }
}

template <int MODE, class RT>
hipError_t launch_first_x_region(const Lattice& lat, Planes3 xout, int sweeps,
                                 unsigned long long* rslot, FirstArgs fa, const Multi& mu,
                                 int region, hipStream_t stream, LaunchEvents ev, PrevStep pv) {
  const CPlanes3 none{{nullptr, nullptr, nullptr}};
  const Planes3 nout{{nullptr, nullptr, nullptr}};
  const ConvCheck nochk{nullptr, 0, 0.0, false};
  if (sizeof(RT) == sizeof(float) && region != kRegion32x32) return hipErrorInvalidValue;
  switch (region) {
    case kRegion32x32:
      return launch_solve_region<32, 32, MODE, RT>(lat, none, nout, xout, rslot, nochk, fa,
                                                   sweeps, mu, stream, ev, pv);
    case kRegion64x16:
      return launch_solve_region<64, 16, MODE, double>(lat, none, nout, xout, rslot, nochk, fa,
                                                       sweeps, mu, stream, ev, pv);
    case kRegion32x16:
      return launch_solve_region<32, 16, MODE, double>(lat, none, nout, xout, rslot, nochk, fa,
                                                       sweeps, mu, stream, ev, pv);
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_stage_solve(const Lattice& lat, CPlanes3 phib, Planes3 rout, int sweeps,
                              unsigned long long* rslot, ConvCheck check, hipStream_t stream,
                              LaunchEvents ev) {
  const Planes3 none{{nullptr, nullptr, nullptr}};
  return launch_solve_region<32, 32, kSolvePlain, double>(lat, phib, none, rout, rslot, check,
                                                          FirstArgs{nullptr, false}, sweeps,
                                                          Multi{}, stream, ev);
}

hipError_t launch_first_solve(const Lattice& lat, Planes3 rout, int sweeps,
                              unsigned long long* rslot, unsigned long long* u0max_slot,
                              Planes3 phib_out, hipStream_t stream, LaunchEvents ev) {
  const CPlanes3 none{{nullptr, nullptr, nullptr}};
  const FirstArgs fa{u0max_slot, phib_out.s[0] != nullptr};
  const ConvCheck nochk{nullptr, 0, 0.0, false};
  return launch_solve_region<32, 32, kSolveFirst, double>(lat, none, phib_out, rout, rslot,
                                                          nochk, fa, sweeps, Multi{}, stream, ev);
}

hipError_t launch_first_solve_x(const Lattice& lat, Planes3 xout, int sweeps,
                                unsigned long long* rslot, unsigned long long* u0max_slot,
                                hipStream_t stream, LaunchEvents ev, const Multi& mu, int region,
                                bool fp32, const PrevStep* prev) {
  const FirstArgs fa{u0max_slot, false};
  if (prev != nullptr)
    return fp32 ? launch_first_x_region<kSolveFirstXPrev, float>(lat, xout, sweeps, rslot, fa, mu,
                                                                 region, stream, ev, *prev)
                : launch_first_x_region<kSolveFirstXPrev, double>(lat, xout, sweeps, rslot, fa,
                                                                  mu, region, stream, ev, *prev);
  return fp32 ? launch_first_x_region<kSolveFirstX, float>(lat, xout, sweeps, rslot, fa, mu,
                                                           region, stream, ev, PrevStep{})
              : launch_first_x_region<kSolveFirstX, double>(lat, xout, sweeps, rslot, fa, mu,
                                                            region, stream, ev, PrevStep{});
}

hipError_t launch_stage_sweep(const Lattice& lat, CPlanes3 phib, CPlanes3 rin, Planes3 rout,
                              unsigned long long* rslot, ConvCheck check, hipStream_t stream,
                              LaunchEvents ev) {
  MB4_LAUNCH(k_stage_sweep, dim3(tile_blocks(lat.nx, lat.ny)), dim3(kTile), ev, lat, phib, rin,
             rout, rslot, check);
}

hipError_t launch_iterate(const Lattice& lat, CPlanes3 Xin, Planes3 Xout, int sweeps,
                          unsigned long long* rnext, ConvCheck check, ConvCheck fin, StepOut so,
                          hipStream_t stream, LaunchEvents ev, const Multi& mu, int region,
                          bool fp32) {
  if (fp32) {
    if (region != kRegion32x32) return hipErrorInvalidValue;
    return launch_iterate_region<32, 32, float>(lat, Xin, Xout, sweeps, rnext, check, fin, so,
                                                mu, stream, ev);
  }
  switch (region) {
    case kRegion32x32:
      return launch_iterate_region<32, 32, double>(lat, Xin, Xout, sweeps, rnext, check, fin, so,
                                                   mu, stream, ev);
    case kRegion64x16:
      return launch_iterate_region<64, 16, double>(lat, Xin, Xout, sweeps, rnext, check, fin, so,
                                                   mu, stream, ev);
    case kRegion32x16:
      return launch_iterate_region<32, 16, double>(lat, Xin, Xout, sweeps, rnext, check, fin, so,
                                                   mu, stream, ev);
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_final_update(const Lattice& lat, CPlanes3 X, ConvCheck check, ConvCheck fin,
                               StepOut so, hipStream_t stream, LaunchEvents ev, const Multi& mu) {
  const int n = lat.nx * lat.ny;
  const dim3 grid(mu.desc != nullptr ? mu.blocks : (n + kFinalSites - 1) / kFinalSites),
      block(kFinalSites);
  MB4_LAUNCH(k_final_update, grid, block, ev, lat, X, check, fin, so, n, mu);
}

namespace {

template <int RX, int RY, class RT>
const void* member_run_kernel(int sweeps) {
  switch (sweeps) {
    case 1:
      return reinterpret_cast<const void*>(&k_member_run<RX, RY, 0, RT>);
    case 2:
      return reinterpret_cast<const void*>(&k_member_run<RX, RY, 1, RT>);
    case 3:
      return reinterpret_cast<const void*>(&k_member_run<RX, RY, 2, RT>);
    case 4:
      return reinterpret_cast<const void*>(&k_member_run<RX, RY, 3, RT>);
    default:
      return nullptr;
  }
}

const void* member_run_kernel(int sweeps, int region, bool fp32) {
  if (fp32) return region == kRegion32x32 ? member_run_kernel<32, 32, float>(sweeps) : nullptr;
  switch (region) {
    case kRegion32x32:
      return member_run_kernel<32, 32, double>(sweeps);
    case kRegion64x16:
      return member_run_kernel<64, 16, double>(sweeps);
    case kRegion32x16:
      return member_run_kernel<32, 16, double>(sweeps);
    default:
      return nullptr;
  }
}

int member_run_threads(int region) {
  return region_threads(region_x(region), region_y(region));
}

}  // namespace

hipError_t launch_member_run(const Lattice& lat, const MemberRun& run, int workers, int sweeps,
                             int region, bool fp32, hipStream_t stream, LaunchEvents ev) {
  const void* fn = member_run_kernel(sweeps, region, fp32);
  if (fn == nullptr || workers < 1) return hipErrorInvalidValue;
  Lattice l = lat;
  MemberRun r = run;
  void* args[] = {&l, &r};
  const dim3 grid(workers), block(member_run_threads(region));
  if (ev.start == nullptr && ev.stop == nullptr) {
    const hipError_t err = hipLaunchKernel(fn, grid, block, args, 0, stream);
    return err != hipSuccess ? err : hipGetLastError();
  }
  if (ev.start != nullptr) {
    const hipError_t err = hipEventRecord(ev.start, stream);
    if (err != hipSuccess) return err;
  }
  hipError_t err = hipLaunchKernel(fn, grid, block, args, 0, stream);
  if (err == hipSuccess && ev.stop != nullptr) err = hipEventRecord(ev.stop, stream);
  return err != hipSuccess ? err : hipGetLastError();
}

int member_run_blocks_per_cu(int sweeps, int region, bool fp32) {
  const void* fn = member_run_kernel(sweeps, region, fp32);
  if (fn == nullptr) return 0;
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, member_run_threads(region), 0) !=
      hipSuccess)
    return 0;
  return n;
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
  hipLaunchKernelGGL(k_energy_partial<false>, dim3(nb), dim3(kTile), 0, stream, lat, partials,
                     Multi{}, PsiPlanes{nullptr, nullptr});
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(kTile), 0, stream,
                     static_cast<const double*>(partials), nb, static_cast<const int*>(nullptr),
                     out);
  return hipGetLastError();
}

hipError_t launch_energy_planes(const Lattice& lat, const double* p, const double* q,
                                double* partials, double* out, hipStream_t stream) {
  const int nb = tile_blocks(lat.nx, lat.ny);
  hipLaunchKernelGGL(k_energy_partial<true>, dim3(nb), dim3(kTile), 0, stream, lat, partials,
                     Multi{}, PsiPlanes{p, q});
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(kTile), 0, stream,
                     static_cast<const double*>(partials), nb, static_cast<const int*>(nullptr),
                     out);
  return hipGetLastError();
}

hipError_t launch_energy_multi(const Lattice& lat, const Multi& mu, double* partials,
                               double* out, hipStream_t stream) {
  hipLaunchKernelGGL(k_energy_partial<false>, dim3(mu.blocks), dim3(kTile), 0, stream, lat,
                     partials, mu, PsiPlanes{nullptr, nullptr});
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_energy_final, dim3(mu.count), dim3(kTile), 0, stream,
                     static_cast<const double*>(partials), mu.blocks, mu.block0, out);
  return hipGetLastError();
}

}  // namespace mb4
