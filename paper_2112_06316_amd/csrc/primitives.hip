// Device-wide primitives used while building a plan: exclusive prefix sums
// and a sort of 64-bit keys.  Plan-time only; none of this runs in an apply.
#include "internal.h"

namespace ifgf {

namespace {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;   // 4096

template <typename TIn>
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_reduce(const TIn* __restrict__ in, int64_t n,
                                                              int* __restrict__ bsum) {
  __shared__ int red[SCAN_THREADS / 64];
  int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
  int acc = 0;
  for (int i = threadIdx.x; i < SCAN_TILE; i += SCAN_THREADS) {
    int64_t g = base + i;
    if (g < n) acc += (int)in[g];
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < SCAN_THREADS / 64; ++w) t += red[w];
    bsum[blockIdx.x] = t;
  }
}

// Exclusive scan of one tile; block offsets from `boff` (may be null).
template <typename TIn>
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_apply(const TIn* __restrict__ in, int64_t n,
                                                             const int* __restrict__ boff,
                                                             int* __restrict__ out) {
  __shared__ int wsum[SCAN_THREADS / 64];
  int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  int v[SCAN_ITEMS];
  int tot = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    int64_t g = base + i;
    v[i] = g < n ? (int)in[g] : 0;
    tot += v[i];
  }
  // inclusive scan of thread totals within the wave
  int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int x = tot;
  for (int off = 1; off < 64; off <<= 1) {
    int y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) wsum[wid] = x;
  __syncthreads();
  int woff = 0;
  for (int w = 0; w < wid; ++w) woff += wsum[w];
  int run = (boff ? boff[blockIdx.x] : 0) + woff + x - tot;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    int64_t g = base + i;
    if (g < n) out[g] = run;
    run += v[i];
  }
  // the thread that owns the last element writes the total at out[n]
  if (base <= n - 1 && n - 1 < base + SCAN_ITEMS) out[n] = run;   // run = total here
}

template <typename TIn>
void scan_impl(const TIn* in, int* out, int64_t n, hipStream_t s) {
  if (n <= 0) {
    HIPCHK(hipMemsetAsync(out, 0, sizeof(int), s));
    return;
  }
  int64_t nblk = (n + SCAN_TILE - 1) / SCAN_TILE;
  if (nblk == 1) {
    k_scan_apply<TIn><<<1, SCAN_THREADS, 0, s>>>(in, n, nullptr, out);
    HIPCHK(hipGetLastError());
    return;
  }
  int* bsum = nullptr;
  HIPCHK(hipMallocAsync((void**)&bsum, sizeof(int) * (nblk + 1), s));
  k_scan_reduce<TIn><<<(unsigned)nblk, SCAN_THREADS, 0, s>>>(in, n, bsum);
  HIPCHK(hipGetLastError());
  // exclusive scan of the block sums, in place into a second buffer
  int* boff = nullptr;
  HIPCHK(hipMallocAsync((void**)&boff, sizeof(int) * (nblk + 1), s));
  scan_impl<int>(bsum, boff, nblk, s);
  k_scan_apply<TIn><<<(unsigned)nblk, SCAN_THREADS, 0, s>>>(in, n, boff, out);
  HIPCHK(hipGetLastError());
  HIPCHK(hipFreeAsync(bsum, s));
  HIPCHK(hipFreeAsync(boff, s));
}

// --------------------------------------------------------------------------
// Bitonic sort of uint64 keys (ascending).  The keys sorted here are unique
// (Morton key in the high word, original index in the low word), so the
// result is the unique sorted order whatever the algorithm's stability.
// --------------------------------------------------------------------------
constexpr int BT_TILE = 2048;
constexpr int BT_THREADS = 1024;

__global__ __launch_bounds__(BT_THREADS) void k_bitonic_local(uint64_t* __restrict__ a, int64_t kmax_stage,
                                                              int full) {
  // full = 1: run every stage k = 2..BT_TILE; full = 0: run the tail j = BT_TILE/2..1
  // of global stage k = kmax_stage.
  __shared__ uint64_t t[BT_TILE];
  int64_t base = (int64_t)blockIdx.x * BT_TILE;
  t[threadIdx.x] = a[base + threadIdx.x];
  t[threadIdx.x + BT_THREADS] = a[base + threadIdx.x + BT_THREADS];
  __syncthreads();
  int64_t k0 = full ? 2 : kmax_stage;
  int64_t k1 = full ? BT_TILE : kmax_stage;
  for (int64_t k = k0; k <= k1; k <<= 1) {
    int jstart = full ? (int)(k >> 1) : BT_TILE / 2;
    for (int j = jstart; j > 0; j >>= 1) {
      int i = 2 * j * (threadIdx.x / j) + (threadIdx.x % j);
      int l = i + j;
      int64_t gi = base + i;
      bool up = (gi & k) == 0;
      uint64_t x = t[i], y = t[l];
      if ((x > y) == up) {
        t[i] = y;
        t[l] = x;
      }
      __syncthreads();
    }
  }
  a[base + threadIdx.x] = t[threadIdx.x];
  a[base + threadIdx.x + BT_THREADS] = t[threadIdx.x + BT_THREADS];
}

__global__ void k_bitonic_global(uint64_t* __restrict__ a, int64_t n2, int64_t k, int64_t j) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n2 / 2) return;
  int64_t i = 2 * j * (t / j) + (t % j);
  int64_t l = i + j;
  bool up = (i & k) == 0;
  uint64_t x = a[i], y = a[l];
  if ((x > y) == up) {
    a[i] = y;
    a[l] = x;
  }
}

__global__ void k_fill_u64(uint64_t* a, int64_t lo, int64_t hi, uint64_t v) {
  int64_t i = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < hi) a[i] = v;
}

}  // namespace

void scan_exclusive_u8(const uint8_t* in, int* out, int64_t n, hipStream_t s) { scan_impl<uint8_t>(in, out, n, s); }
void scan_exclusive_i32(const int* in, int* out, int64_t n, hipStream_t s) { scan_impl<int>(in, out, n, s); }

// Sorts data[0..n) ascending.  `data` must have room for the padded length
// (next power of two >= max(n, 2048)); see sort_padded_length().
int64_t sort_padded_length(int64_t n) {
  int64_t n2 = BT_TILE;
  while (n2 < n) n2 <<= 1;
  return n2;
}

void sort_u64(uint64_t* data, int64_t n, hipStream_t s) {
  int64_t n2 = sort_padded_length(n);
  if (n2 > n) {
    int64_t cnt = n2 - n;
    k_fill_u64<<<(unsigned)((cnt + 255) / 256), 256, 0, s>>>(data, n, n2, ~0ull);
    HIPCHK(hipGetLastError());
  }
  unsigned tiles = (unsigned)(n2 / BT_TILE);
  k_bitonic_local<<<tiles, BT_THREADS, 0, s>>>(data, 0, 1);
  HIPCHK(hipGetLastError());
  for (int64_t k = 2 * BT_TILE; k <= n2; k <<= 1) {
    for (int64_t j = k >> 1; j >= BT_TILE; j >>= 1) {
      int64_t th = n2 / 2;
      k_bitonic_global<<<(unsigned)((th + 255) / 256), 256, 0, s>>>(data, n2, k, j);
      HIPCHK(hipGetLastError());
    }
    k_bitonic_local<<<tiles, BT_THREADS, 0, s>>>(data, k, 0);
    HIPCHK(hipGetLastError());
  }
}

}  // namespace ifgf
