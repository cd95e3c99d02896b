// Interface detection that allocates nothing (dcm_detect_interface_noalloc),
// for callers that cannot allocate device memory: code under HIP graph
// capture, tight serving loops, harnesses that forbid allocation.
//
// Its scratch -- the histogram copies, the gray values, the two bit-packed
// phase maps and, when the caller passes no counts array, the voxel counts --
// lives in one static device array per GPU instead of context-owned buffers.
// In host code the array's name is only a host-side stand-in, so its device
// address is looked up once per device (hipGetSymbolAddress, with that device
// current, when a context is created on it) and only that address is ever
// handed to kernels.  Every call on a GPU shares the array and leaves its
// contents behind: the detection clears what must start at zero (counts and
// histograms, with fill kernels), and calls that overlap on one GPU race.
#include <mutex>

#include "dcm_internal.hpp"

namespace dcm {

namespace {

constexpr size_t kScratchBytes = size_t(32) << 20;  // 32 MiB per GPU
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
unsigned char *g_scratch[kMaxDevices] = {};  // device address per device (null: not looked up)

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

dcm_status noalloc_scratch_setup(int device, std::string *err) {
  if (device < 0 || device >= kMaxDevices) {
    if (err) *err = "device index beyond the no-allocation scratch table";
    return DCM_ERR_HIP;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_scratch[device]) return DCM_OK;
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != device) {
    (void)hipGetLastError();  // clear the sticky error
    if (err) *err = "no-allocation scratch: the context's device is not current";
    return DCM_ERR_HIP;
  }
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();  // clear the sticky error
    if (err) *err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
    return DCM_ERR_HIP;
  }
  g_scratch[device] = static_cast<unsigned char *>(p);
  return DCM_OK;
}

}  // namespace dcm

using namespace dcm;

extern "C" dcm_status dcm_detect_interface_noalloc(dcm_ctx *ctx, const double *x,
                                                   const double *y, const double *z, int64_t n,
                                                   dcm_box box, dcm_grid grid, double split,
                                                   uint32_t *counts, uint8_t *seg,
                                                   uint8_t *iface, int32_t *threshold_out) {
  const dcm_detect_opts opts = {split, -1.0, 0};
  int64_t nvox = 0;
  dcm_status st = detect_check(ctx, x, y, z, n, box, grid, &opts, seg, iface, &nvox);
  if (st != DCM_OK) return st;
  unsigned char *base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    if (ctx->device >= 0 && ctx->device < kMaxDevices) base = g_scratch[ctx->device];
  }
  if (!base) return fail(ctx, DCM_ERR_HIP, "no-allocation scratch was not set up on this device");
  // layout: histogram copies, gray values, phase maps, counts (if needed)
  const size_t hist_b = align256((size_t)kHistCopies * kHistBins * sizeof(uint32_t));
  const size_t gray_b = align256((size_t)nvox * sizeof(uint32_t));
  const size_t map_b = align256((size_t)phase_bits_words(grid.n) * sizeof(uint32_t));
  const size_t counts_b = counts ? 0 : gray_b;
  const size_t need = hist_b + gray_b + 2 * map_b + counts_b;
  if (need > kScratchBytes)
    return fail(ctx, DCM_ERR_RANGE,
                "dcm_detect_interface_noalloc: the grid needs " + std::to_string(need) +
                    " scratch bytes, more than its fixed " + std::to_string(kScratchBytes));
  DetectScratch sc;
  sc.hist = reinterpret_cast<uint32_t *>(base);
  sc.gray = reinterpret_cast<uint32_t *>(base + hist_b);
  sc.seg_a = reinterpret_cast<uint32_t *>(base + hist_b + gray_b);
  sc.seg_b = reinterpret_cast<uint32_t *>(base + hist_b + gray_b + map_b);
  sc.counts = counts ? counts : reinterpret_cast<uint32_t *>(base + hist_b + gray_b + 2 * map_b);
  return detect_enqueue(ctx, x, y, z, n, box, grid, opts, sc, seg, iface, threshold_out, false);
}
