// Batched projection onto second-order cones (supplementary II-C).
//
// Memory-bound: each entry is read once and written once.  A workgroup owns
// the cones whose first entry (t) falls in its tile of TILE entries; their
// entries are streamed with coalesced loads into LDS (up to CAP), the squared
// norms of the eta parts are reduced per cone in a fixed order (one thread per
// short cone, one wave per long cone), and a second sweep over the staged
// values applies the closed form:
//   a = ||eta||;  a <= t -> unchanged;  a <= -t -> 0;  else ((t+a)/2, (t+a)/(2a) eta).
// Entries of an owned cone beyond CAP (cones longer than CAP - TILE) are read
// from global memory a second time.
#include <mutex>
#include <string>

#include "common.hpp"
#include "internal.hpp"

namespace nrto {

constexpr int PS_THREADS = 256;
constexpr int PS_TILE = 1024;
constexpr int PS_CAP = 4096;
constexpr int PS_SHORT = 32;   // cones with more eta entries are reduced by a wave

__device__ __forceinline__ int64_t lower_bound_i64(const int64_t* a, int64_t n, int64_t key) {
  // first index i in [0, n] with a[i] >= key (a has n + 1 readable entries)
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1; else hi = mid;
  }
  return lo;
}

template <typename F>
__global__ void __launch_bounds__(PS_THREADS)
project_soc_kernel(const F* in, F* out, const int64_t* __restrict__ off,
                   int64_t ncones, int64_t N) {
  __shared__ F stage[PS_CAP];
  __shared__ double sums[PS_TILE];
  __shared__ int32_t coff[PS_TILE + 1];
  __shared__ int64_t range[2];

  const int64_t tile_lo = (int64_t)blockIdx.x * PS_TILE;
  const int64_t tile_hi = min(tile_lo + (int64_t)PS_TILE, N);
  if (threadIdx.x == 0) {
    range[0] = lower_bound_i64(off, ncones, tile_lo);
    range[1] = lower_bound_i64(off, ncones, tile_hi);
  }
  __syncthreads();
  const int64_t cb_all = range[0], ce_all = range[1];
  // Cones starting in this tile, in chunks of at most TILE cones (more only with empty cones).
  for (int64_t cb = cb_all; cb < ce_all; cb += PS_TILE) {
    const int64_t ce = min(cb + (int64_t)PS_TILE, ce_all);
    const int nown = (int)(ce - cb);
    const int64_t e_lo = min(max(off[cb], (int64_t)0), N);
    const int64_t e_hi = min(max(off[ce], e_lo), N);
    const int64_t len = e_hi - e_lo;
    for (int i = threadIdx.x; i <= nown; i += PS_THREADS) {
      int64_t o = min(max(off[cb + i], e_lo), e_hi);
      coff[i] = (int32_t)min(o - e_lo, (int64_t)0x7fffffff);
    }
    __syncthreads();
    // phase 1: stage the tile's entries
    for (int64_t l = threadIdx.x; l < len && l < PS_CAP; l += PS_THREADS) stage[l] = in[e_lo + l];
    __syncthreads();
    // ||eta||^2 per owned cone in a fixed summation order (the result does not
    // depend on scheduling): a cone with at most SHORT eta entries is summed
    // serially by one thread, a longer one by one wave (lane-strided partial
    // sums, then a butterfly over the lanes)
    for (int i = threadIdx.x; i < nown; i += PS_THREADS) {
      const int c0 = coff[i], c1 = coff[i + 1];
      if (c1 - c0 - 1 <= PS_SHORT) {
        double acc = 0.0;
        for (int l = c0 + 1; l < c1; ++l) {
          const double v = (double)((l < PS_CAP) ? stage[l] : in[e_lo + l]);
          acc += v * v;
        }
        sums[i] = acc;
      }
    }
    for (int i = wave_id(); i < nown; i += PS_THREADS / NRTO_WAVE) {
      const int c0 = coff[i], c1 = coff[i + 1];
      if (c1 - c0 - 1 > PS_SHORT) {
        double acc = 0.0;
        for (int l = c0 + 1 + lane_id(); l < c1; l += NRTO_WAVE) {
          const double v = (double)((l < PS_CAP) ? stage[l] : in[e_lo + l]);
          acc += v * v;
        }
        acc = wave_sum(acc);
        if (lane_id() == 0) sums[i] = acc;
      }
    }
    __syncthreads();
    // phase 2: closed-form projection
    for (int64_t l = threadIdx.x; l < len; l += PS_THREADS) {
      int lo = 0, hi = nown - 1;
      while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (coff[mid] <= l) lo = mid; else hi = mid - 1;
      }
      const int c0 = coff[lo];
      const double t = (double)((c0 < PS_CAP) ? stage[c0] : in[e_lo + c0]);
      const double a = sqrt(sums[lo]);
      F v = (l < PS_CAP) ? stage[l] : in[e_lo + l];
      double r;
      if (a <= t) {
        r = (double)v;
      } else if (a <= -t) {
        r = 0.0;
      } else {
        const double sc = 0.5 * (t + a);
        r = (l == c0) ? sc : (sc / a) * (double)v;
      }
      out[e_lo + l] = (F)r;
    }
    __syncthreads();
  }
}

__global__ void validate_offsets_kernel(const int64_t* off, int64_t ncones, int64_t N, int* bad) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0 && (off[0] != 0 || off[ncones] != N)) atomicOr(bad, 1);
  if (i < ncones && off[i + 1] < off[i]) atomicOr(bad, 1);
}

// Scratch of nrto_project_soc_noalloc: word 0 is the offset-validation flag,
// the other words are unused.  Every device the library runs on holds its own
// copy for the life of the process; host code reaches it only through the
// address hipGetSymbolAddress returns for the current device.
constexpr int NOALLOC_SCRATCH_WORDS = 64;
static __device__ __align__(256) int32_t scratch[NOALLOC_SCRATCH_WORDS];

__global__ void clear_words_kernel(int32_t* w, int n) {
  if ((int)threadIdx.x < n) w[threadIdx.x] = 0;
}

constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static int32_t* g_scratch_dev[NOALLOC_MAX_DEVICES] = {};

// Device address of `scratch` on the current device, resolved once per device.
static nrto_status scratch_address(int32_t** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return set_global_error(NRTO_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
    return set_global_error(NRTO_ERR_ARG, "device ordinal beyond the 64 devices the scratch table covers");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_global_error(NRTO_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_dev[dev] = (int32_t*)p;
  }
  *out = g_scratch_dev[dev];
  return NRTO_OK;
}

}  // namespace nrto

using namespace nrto;

static nrto_status launch_projection(const void* in, void* out, const int64_t* seg_off, int64_t n_cones,
                                     int64_t n_entries, int32_t dtype, hipStream_t s) {
  int64_t nblocks = (n_entries + PS_TILE - 1) / PS_TILE;
  if (nblocks > 0x7fffffff) return set_global_error(NRTO_ERR_ARG, "too many entries");
  if (dtype == 0)
    project_soc_kernel<double><<<dim3((unsigned)nblocks), dim3(PS_THREADS), 0, s>>>(
        (const double*)in, (double*)out, seg_off, n_cones, n_entries);
  else
    project_soc_kernel<float><<<dim3((unsigned)nblocks), dim3(PS_THREADS), 0, s>>>(
        (const float*)in, (float*)out, seg_off, n_cones, n_entries);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_global_error(NRTO_ERR_HIP, hipGetErrorString(e));
  return NRTO_OK;
}

extern "C" nrto_status nrto_project_soc(const void* in, void* out, const int64_t* seg_off,
                                        int64_t n_cones, int64_t n_entries, int32_t dtype,
                                        int32_t flags, void* stream) {
  if (n_cones < 0 || n_entries < 0) return set_global_error(NRTO_ERR_ARG, "negative size");
  if (dtype != 0 && dtype != 1) return set_global_error(NRTO_ERR_ARG, "dtype must be 0 (f64) or 1 (f32)");
  if (n_entries == 0 || n_cones == 0) return NRTO_OK;
  if (!in || !out || !seg_off) return set_global_error(NRTO_ERR_ARG, "null pointer");
  hipStream_t s = (hipStream_t)stream;
  if (flags & 1) {
    int* bad = nullptr;
    if (hipMalloc(&bad, sizeof(int)) != hipSuccess) return set_global_error(NRTO_ERR_ALLOC, "hipMalloc failed");
    int zero = 0, h = 0;
    hipError_t e = hipMemcpyAsync(bad, &zero, sizeof(int), hipMemcpyHostToDevice, s);
    int64_t nb = (n_cones + 255) / 256;
    if (e == hipSuccess) {
      validate_offsets_kernel<<<dim3((unsigned)nb), dim3(256), 0, s>>>(seg_off, n_cones, n_entries, bad);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(&h, bad, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(bad);
    if (e != hipSuccess) return set_global_error(NRTO_ERR_HIP, hipGetErrorString(e));
    if (h) return set_global_error(NRTO_ERR_ARG, "seg_off must start at 0, be non-decreasing and end at n_entries");
  }
  return launch_projection(in, out, seg_off, n_cones, n_entries, dtype, s);
}

extern "C" nrto_status nrto_project_soc_noalloc(const void* in, void* out, const int64_t* seg_off,
                                                int64_t n_cones, int64_t n_entries, int32_t dtype,
                                                void* stream) {
  if (n_cones < 0 || n_entries < 0) return set_global_error(NRTO_ERR_ARG, "negative size");
  if (dtype != 0 && dtype != 1) return set_global_error(NRTO_ERR_ARG, "dtype must be 0 (f64) or 1 (f32)");
  if (n_entries == 0 || n_cones == 0) return NRTO_OK;
  if (!in || !out || !seg_off) return set_global_error(NRTO_ERR_ARG, "null pointer");
  if ((n_cones + 255) / 256 > 0x7fffffff || (n_entries + PS_TILE - 1) / PS_TILE > 0x7fffffff)
    return set_global_error(NRTO_ERR_ARG, "too many cones or entries for one launch");
  int32_t* scr = nullptr;
  nrto_status st = scratch_address(&scr);
  if (st != NRTO_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  // the flag keeps the previous call's value: clear it with a kernel (no memset node)
  clear_words_kernel<<<dim3(1), dim3(64), 0, s>>>(scr, 1);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) {
    validate_offsets_kernel<<<dim3((unsigned)((n_cones + 255) / 256)), dim3(256), 0, s>>>(seg_off, n_cones,
                                                                                      n_entries, scr);
    e = hipGetLastError();
  }
  int32_t h = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&h, scr, sizeof(int32_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return set_global_error(NRTO_ERR_HIP, hipGetErrorString(e));
  if (h) return set_global_error(NRTO_ERR_ARG, "seg_off must start at 0, be non-decreasing and end at n_entries");
  return launch_projection(in, out, seg_off, n_cones, n_entries, dtype, s);
}
