// Device-wide exclusive scan and stable LSD radix sort (4-bit digits) for the
// tree build.  Tiles of 2048 elements: 256 threads with 8 consecutive elements
// each, so that a tile's order is thread order, then item order.  Per-tile
// counts and sums go through LDS; the global offsets come from a scan of the
// per-(digit, tile) counts in digit-major order, which is what makes the sort
// stable.  No global atomics: the results do not depend on scheduling.
#include "sort_scan.hpp"

namespace tefmm {

namespace {

constexpr int BT = 256, IT = 8, TILE = BT * IT;
constexpr int RB = 4, NBIN = 1 << RB;

inline int64_t tiles(int64_t n) { return (n + TILE - 1) / TILE; }
inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// exclusive scan of the 256 per-thread values v[t] in LDS buffer sh (256 entries);
// returns this thread's exclusive prefix, *total the block's sum
__device__ unsigned block_exclusive(unsigned v, unsigned* sh, unsigned* total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < BT; off <<= 1) {
    const unsigned a = t >= off ? sh[t - off] : 0u;
    __syncthreads();
    sh[t] += a;
    __syncthreads();
  }
  const unsigned incl = sh[t];
  *total = sh[BT - 1];
  __syncthreads();
  return incl - v;
}

// out[i] = exclusive prefix of in within the tile; sums[tile] = the tile's total
__global__ __launch_bounds__(BT) void k_scan_tile(const unsigned* in, unsigned* out, int64_t n, unsigned* sums) {
  __shared__ unsigned sh[BT];
  const int64_t base = (int64_t)blockIdx.x * TILE + (int64_t)threadIdx.x * IT;
  unsigned v[IT], tot = 0;
#pragma unroll
  for (int j = 0; j < IT; ++j) {
    v[j] = base + j < n ? in[base + j] : 0u;
    tot += v[j];
  }
  unsigned btot;
  unsigned run = block_exclusive(tot, sh, &btot);
#pragma unroll
  for (int j = 0; j < IT; ++j) {
    if (base + j < n) out[base + j] = run;
    run += v[j];
  }
  if (threadIdx.x == 0 && sums) sums[blockIdx.x] = btot;
}

// out[i] += offs[tile of i]
__global__ __launch_bounds__(BT) void k_scan_add(unsigned* out, int64_t n, const unsigned* offs) {
  const int64_t base = (int64_t)blockIdx.x * TILE + (int64_t)threadIdx.x * IT;
  const unsigned o = offs[blockIdx.x];
#pragma unroll
  for (int j = 0; j < IT; ++j)
    if (base + j < n) out[base + j] += o;
}

// digit counts of this thread's 8 keys, packed 4 bits per digit value (at most 8 each)
__device__ __forceinline__ unsigned long long digit_counts(const unsigned* keys, int64_t base, int64_t n, int shift) {
  unsigned long long c = 0;
#pragma unroll
  for (int j = 0; j < IT; ++j)
    if (base + j < n) c += 1ull << (RB * ((keys[base + j] >> shift) & (NBIN - 1)));
  return c;
}

// hist[d * ntiles + tile] = keys of digit d in the tile
__global__ __launch_bounds__(BT) void k_radix_count(const unsigned* keys, int64_t n, int shift, unsigned* hist,
                                                    int64_t ntiles) {
  __shared__ unsigned cnt[NBIN][BT];
  const int t = threadIdx.x;
  const unsigned long long c = digit_counts(keys, (int64_t)blockIdx.x * TILE + (int64_t)t * IT, n, shift);
#pragma unroll
  for (int d = 0; d < NBIN; ++d) cnt[d][t] = (unsigned)((c >> (RB * d)) & (NBIN - 1));
  __syncthreads();
  if (t < NBIN) {
    unsigned s = 0;
    for (int i = 0; i < BT; ++i) s += cnt[t][i];
    hist[(int64_t)t * ntiles + blockIdx.x] = s;
  }
}

// scatter by the scanned counts: key j of thread t with digit d goes to
// offs[d * ntiles + tile] + (keys of digit d in earlier threads of the tile) + (earlier in t)
__global__ __launch_bounds__(BT) void k_radix_scatter(const unsigned* kin, const int* vin, int64_t n, int shift,
                                                      const unsigned* offs, int64_t ntiles, unsigned* kout,
                                                      int* vout) {
  __shared__ unsigned cnt[NBIN][BT + 1];
  const int t = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * TILE + (int64_t)t * IT;
  const unsigned long long c = digit_counts(kin, base, n, shift);
#pragma unroll
  for (int d = 0; d < NBIN; ++d) cnt[d][t] = (unsigned)((c >> (RB * d)) & (NBIN - 1));
  __syncthreads();
  if (t < NBIN) {  // exclusive prefix over the threads, one digit value per thread
    unsigned s = 0;
    for (int i = 0; i < BT; ++i) {
      const unsigned v = cnt[t][i];
      cnt[t][i] = s;
      s += v;
    }
  }
  __syncthreads();
  unsigned long long run = 0;  // keys of each digit value taken so far by this thread (4 bits each)
#pragma unroll
  for (int j = 0; j < IT; ++j) {
    if (base + j >= n) break;
    const unsigned key = kin[base + j];
    const int d = (key >> shift) & (NBIN - 1);
    const unsigned r = (unsigned)((run >> (RB * d)) & (NBIN - 1));
    run += 1ull << (RB * d);
    const int64_t dst = (int64_t)offs[(int64_t)d * ntiles + blockIdx.x] + cnt[d][t] + r;
    kout[dst] = key;
    vout[dst] = vin[base + j];
  }
}

}  // namespace

size_t scan_scratch_bytes(int64_t n) {
  size_t b = 0;
  for (int64_t m = tiles(n); m > 1; m = tiles(m)) b += align256(sizeof(unsigned) * m);
  return b + 256;
}

hipError_t exclusive_scan(const unsigned* in, unsigned* out, int64_t n, void* scratch, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t nt = tiles(n);
  unsigned* sums = nt > 1 ? (unsigned*)scratch : nullptr;
  hipLaunchKernelGGL(k_scan_tile, dim3((unsigned)nt), dim3(BT), 0, s, in, out, n, sums);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || nt == 1) return e;
  // the tile sums, scanned in place with the rest of the scratch, then added back
  void* rest = (char*)scratch + align256(sizeof(unsigned) * nt);
  e = exclusive_scan(sums, sums, nt, rest, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nt), dim3(BT), 0, s, out, n, (const unsigned*)sums);
  return hipGetLastError();
}

size_t sort_scratch_bytes(int64_t n) {
  const int64_t h = NBIN * tiles(n);
  return align256(sizeof(unsigned) * h) + scan_scratch_bytes(h);
}

hipError_t radix_sort_pairs(unsigned* keys_in, unsigned* keys_out, int* vals_in, int* vals_out, int64_t n,
                            int end_bit, void* scratch, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t nt = tiles(n), nh = NBIN * nt;
  unsigned* hist = (unsigned*)scratch;
  void* sc = (char*)scratch + align256(sizeof(unsigned) * nh);
  const int passes = end_bit <= 0 ? 0 : (end_bit + RB - 1) / RB;
  unsigned* ka = keys_in;
  unsigned* kb = keys_out;
  int* va = vals_in;
  int* vb = vals_out;
  for (int p = 0; p < passes; ++p) {
    const int shift = p * RB;
    hipLaunchKernelGGL(k_radix_count, dim3((unsigned)nt), dim3(BT), 0, s, (const unsigned*)ka, n, shift, hist, nt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = exclusive_scan(hist, hist, nh, sc, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nt), dim3(BT), 0, s, (const unsigned*)ka, (const int*)va, n,
                       shift, (const unsigned*)hist, nt, kb, vb);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    std::swap(ka, kb), std::swap(va, vb);
  }
  if (ka != keys_out) {  // an even number of passes (or none) leaves the result in the input buffers
    hipError_t e = hipMemcpyAsync(keys_out, ka, sizeof(unsigned) * n, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(vals_out, va, sizeof(int) * n, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace tefmm
