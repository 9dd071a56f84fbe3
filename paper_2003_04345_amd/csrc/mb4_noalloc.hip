// Energy components of a device field without any allocation
// (mb4_energy_components_noalloc in include/mb4.h).
//
// The per-block partial sums that mb4_energy_components keeps in its state
// live here in one file-scope device array, `scratch`, of a fixed size.
// Each GPU holds its own copy; host code never passes the array's name to a
// kernel (on the host it is only a stand-in for the symbol), but the device
// address that hipGetSymbolAddress returns for the current device, looked up
// once per device and kept.
#include <math.h>

#include <mutex>

#include "mb4.h"
#include "mb4_internal.h"

namespace {

// Largest number of energy tiles (64 x 4 sites each) a call may cover:
// 8,388,608 sites of full tiles, e.g. 2048 x 4096.
constexpr int kMaxTiles = 32768;
constexpr size_t kScratchDoubles = size_t(kMaxTiles) * 12;  // 6 (hi, lo) pairs per tile

static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on the current device.
int scratch_address(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess)
    return mb4::rt::fail(MB4_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices)
    return mb4::rt::fail(MB4_EDEVICE, "device %d is beyond the %d this library tracks", dev,
                         kMaxDevices);
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_scratch[dev] == nullptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
      return mb4::rt::fail(MB4_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                           hipGetErrorString(e));
    g_scratch[dev] = static_cast<double*>(p);
  }
  *out = g_scratch[dev];
  return MB4_OK;
}

}  // namespace

extern "C" MB4_API int mb4_energy_components_noalloc(const mb4_lattice* lattice,
                                                     const mb4_nonlinearity* nonlinearity,
                                                     const double* d_potential, const double* d_p,
                                                     const double* d_q, double* d_out,
                                                     void* stream) {
  using mb4::rt::fail;
  if (lattice == nullptr || nonlinearity == nullptr)
    return fail(MB4_EINVAL, "lattice and nonlinearity must not be NULL");
  if (d_potential == nullptr || d_p == nullptr || d_q == nullptr || d_out == nullptr)
    return fail(MB4_EINVAL, "d_potential, d_p, d_q and d_out must not be NULL");
  const int nx = lattice->nx, ny = lattice->ny;
  if (nx < 3 || ny < 3) return fail(MB4_EINVAL, "lattice %d x %d: both sides must be >= 3", nx, ny);
  if (int64_t(nx) * int64_t(ny) > (int64_t(1) << 28))
    return fail(MB4_EINVAL, "lattice %d x %d has more than 2^28 sites", nx, ny);
  if (!isfinite(lattice->t_hop) || !isfinite(lattice->diag_shift) || !isfinite(nonlinearity->g))
    return fail(MB4_EINVAL, "t_hop, diag_shift and g must be finite");
  const size_t need = mb4::energy_partials_count(nx, ny);
  if (need > kScratchDoubles)
    return fail(MB4_EINVAL,
                "lattice %d x %d needs %zu energy tiles; the preallocated scratch holds %d",
                nx, ny, need / 12, kMaxTiles);
  double* partials = nullptr;
  const int rc = scratch_address(&partials);
  if (rc != MB4_OK) return rc;
  mb4::Lattice L;
  L.nx = nx;
  L.ny = ny;
  L.t = lattice->t_hop;
  L.shift = lattice->diag_shift;
  L.g = nonlinearity->g;
  L.h = 0.0;
  L.V = d_potential;
  L.u0 = nullptr;
  const hipError_t e = mb4::launch_energy_planes(L, d_p, d_q, partials, d_out,
                                                 static_cast<hipStream_t>(stream));
  if (e != hipSuccess)
    return fail(MB4_EDEVICE, "energy kernels: %s", hipGetErrorString(e));
  return MB4_OK;
}
