// Exclusive prefix sums into int64 (the prefix-sum building block of the
// fine- and coarse-level algorithms, Section 3.2 / 3.3): reduce-then-scan over
// blocks of 2048 elements, recursing on the block sums.
#include "common.h"
#include "kernels.h"

namespace mg {

constexpr int SCAN_BS = 256;
constexpr int SCAN_IPT = 8;
constexpr int SCAN_ITEMS = SCAN_BS * SCAN_IPT;

// Block-wide exclusive scan of one value per thread; returns the block total.
MG_INLINE int64_t block_excl_scan(int64_t v, int64_t* sh_wave, int64_t& total) {
  const int t = threadIdx.x, w = t / MG_WAVE, nw = blockDim.x / MG_WAVE;
  int64_t inc = wave_incl_scan(v);
  if (lane() == MG_WAVE - 1) sh_wave[w] = inc;
  __syncthreads();
  int64_t before = 0;
  total = 0;
  for (int k = 0; k < nw; ++k) {
    int64_t s = sh_wave[k];
    if (k < w) before += s;
    total += s;
  }
  __syncthreads();
  return before + inc - v;
}

template <typename Tin>
__global__ void __launch_bounds__(SCAN_BS) k_scan_blocks(const Tin* __restrict__ in, int64_t* out,
                                                          int64_t n, int64_t* block_sums,
                                                          const int64_t* carry, int64_t* total_out) {
  __shared__ int64_t sh[SCAN_ITEMS];
  __shared__ int64_t sh_wave[SCAN_BS / MG_WAVE];
  const int64_t base = (int64_t)blockIdx.x * SCAN_ITEMS;
  const int t = threadIdx.x;
#pragma unroll
  for (int k = 0; k < SCAN_IPT; ++k) {
    int64_t i = base + t + k * SCAN_BS;
    sh[t + k * SCAN_BS] = (i < n) ? (int64_t)in[i] : 0;
  }
  __syncthreads();
  int64_t loc[SCAN_IPT];
  int64_t s = 0;
#pragma unroll
  for (int k = 0; k < SCAN_IPT; ++k) {
    loc[k] = s;
    s += sh[t * SCAN_IPT + k];
  }
  int64_t tot;
  int64_t off = block_excl_scan(s, sh_wave, tot);
  const int64_t c = (carry && gridDim.x == 1) ? *carry : 0;
#pragma unroll
  for (int k = 0; k < SCAN_IPT; ++k) sh[t * SCAN_IPT + k] = loc[k] + off + c;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < SCAN_IPT; ++k) {
    int64_t i = base + t + k * SCAN_BS;
    if (i < n) out[i] = sh[t + k * SCAN_BS];
  }
  if (t == 0) {
    if (block_sums) block_sums[blockIdx.x] = tot;
    if (gridDim.x == 1 && total_out) *total_out = tot + c;
  }
}

// block_off already includes the carry (it came out of the recursive scan)
__global__ void __launch_bounds__(SCAN_BS) k_scan_add(int64_t* out, int64_t n,
                                                       const int64_t* block_off) {
  const int64_t base = (int64_t)blockIdx.x * SCAN_ITEMS;
  const int64_t add = block_off[blockIdx.x];
#pragma unroll
  for (int k = 0; k < SCAN_IPT; ++k) {
    int64_t i = base + threadIdx.x + k * SCAN_BS;
    if (i < n) out[i] += add;
  }
}

__global__ void k_set_total(int64_t* dst, const int64_t* carry) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = carry ? *carry : 0;
}

size_t scan_temp_bytes(int64_t n) {
  size_t t = 0;
  while (n > SCAN_ITEMS) {
    n = (n + SCAN_ITEMS - 1) / SCAN_ITEMS;
    t += (size_t)n * sizeof(int64_t);
  }
  return t + 2 * sizeof(int64_t);
}

template <typename Tin>
static hipError_t scan_rec(const Tin* in, int64_t* out, int64_t n, int64_t* total,
                           const int64_t* carry, int64_t* temp, hipStream_t st) {
  if (n <= 0) {
    if (total) hipLaunchKernelGGL(k_set_total, 1, 1, 0, st, total, carry);
    return hipGetLastError();
  }
  const int64_t nb = (n + SCAN_ITEMS - 1) / SCAN_ITEMS;
  if (nb == 1) {
    hipLaunchKernelGGL((k_scan_blocks<Tin>), 1, SCAN_BS, 0, st, in, out, n, (int64_t*)nullptr,
                       carry, total);
    return hipGetLastError();
  }
  int64_t* bs = temp;
  hipLaunchKernelGGL((k_scan_blocks<Tin>), (unsigned)nb, SCAN_BS, 0, st, in, out, n, bs,
                     (const int64_t*)nullptr, (int64_t*)nullptr);
  hipError_t e = scan_rec<int64_t>(bs, bs, nb, total, carry, temp + nb, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan_add, (unsigned)nb, SCAN_BS, 0, st, out, n, (const int64_t*)bs);
  return hipGetLastError();
}

hipError_t scan_excl_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* total,
                         const int64_t* carry, void* temp, hipStream_t st) {
  return scan_rec<int64_t>(in, out, n, total, carry, (int64_t*)temp, st);
}
hipError_t scan_excl_i32(const int32_t* in, int64_t* out, int64_t n, int64_t* total,
                         const int64_t* carry, void* temp, hipStream_t st) {
  return scan_rec<int32_t>(in, out, n, total, carry, (int64_t*)temp, st);
}

}  // namespace mg
