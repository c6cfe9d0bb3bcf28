// prim.hip -- device primitives for gfx950 (wave64): exclusive scan of u32
// and a stable LSD radix sort of (u64 key, u32 value) pairs.
//
// The radix sort ranks keys inside a block with wavefront ballots: the lanes
// holding the same 8-bit digit are found with 8 ballots (one per digit bit),
// a lane's rank is the popcount of that mask below it, and per-wave digit
// counts are combined in LDS in wave order.  Items are taken in (round,
// wave, lane) order, so the sort is stable and fully deterministic (no
// ordering depends on atomics).
#include "dem_internal.hpp"

namespace dem {

namespace {

constexpr int kBlock = 256;           // 4 wavefronts of 64
constexpr int kWaves = kBlock / 64;
constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;
constexpr int kSortItems = 8;
constexpr int kSortTile = kBlock * kSortItems;

__device__ inline uint32_t wave_inclusive_scan(uint32_t v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t y = __shfl_up(v, off, 64);
        if (lane >= off) v += y;
    }
    return v;
}

// Exclusive scan of one value per thread over the block; returns the block total in *total.
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t* total)
{
    __shared__ uint32_t wave_tot[kWaves];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    uint32_t inc = wave_inclusive_scan(v);
    if (lane == 63) wave_tot[wave] = inc;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        uint32_t t = wave_tot[w];
        if (w < wave) before += t;
        all += t;
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

__global__ void __launch_bounds__(kBlock) k_scan_reduce(const uint32_t* __restrict__ in, int n,
                                                        uint32_t* __restrict__ sums)
{
    const long base = (long)blockIdx.x * kScanTile;
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        long i = base + (long)k * kBlock + threadIdx.x;
        if (i < n) s += in[i];
    }
    uint32_t total;
    block_exclusive_scan(s, &total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// One block scans the per-tile sums in place, in chunks of kBlock.
__global__ void __launch_bounds__(kBlock) k_scan_top(uint32_t* __restrict__ sums, int nsums,
                                                     uint32_t* __restrict__ total_dev)
{
    uint32_t carry = 0;
    for (int c = 0; c < nsums; c += kBlock) {
        int i = c + threadIdx.x;
        uint32_t v = i < nsums ? sums[i] : 0u;
        uint32_t tot;
        uint32_t ex = block_exclusive_scan(v, &tot);
        if (i < nsums) sums[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0 && total_dev) *total_dev = carry;
}

// Each thread scans kScanItems consecutive elements; in == out is allowed.
__global__ void __launch_bounds__(kBlock) k_scan_down(const uint32_t* in, uint32_t* out, int n,
                                                      const uint32_t* __restrict__ sums)
{
    const long base = (long)blockIdx.x * kScanTile + (long)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        long i = base + k;
        v[k] = i < n ? in[i] : 0u;
        s += v[k];
    }
    uint32_t total;
    uint32_t run = block_exclusive_scan(s, &total) + sums[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        long i = base + k;
        if (i < n) out[i] = run;
        run += v[k];
    }
}

__global__ void __launch_bounds__(kBlock) k_radix_hist(const uint64_t* __restrict__ keys, int n, int shift,
                                                       uint32_t* __restrict__ counts, int nblk)
{
    __shared__ uint32_t hist[256];
    hist[threadIdx.x] = 0;
    __syncthreads();
    const long base = (long)blockIdx.x * kSortTile;
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        long i = base + (long)r * kBlock + threadIdx.x;
        if (i < n) atomicAdd(&hist[(uint32_t)(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    counts[(long)threadIdx.x * nblk + blockIdx.x] = hist[threadIdx.x];
}

__global__ void __launch_bounds__(kBlock) k_radix_scatter(const uint64_t* __restrict__ keys,
                                                          const uint32_t* __restrict__ vals,
                                                          uint64_t* __restrict__ keys_out,
                                                          uint32_t* __restrict__ vals_out, int n, int shift,
                                                          const uint32_t* __restrict__ offsets, int nblk)
{
    __shared__ uint32_t base[256];
    __shared__ uint32_t wcount[kWaves][256];
    __shared__ uint32_t woff[kWaves][256];
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wave = t >> 6;
    base[t] = offsets[(long)t * nblk + blockIdx.x];
    const long tile = (long)blockIdx.x * kSortTile;
    const unsigned long long lanes_below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int r = 0; r < kSortItems; ++r) {
#pragma unroll
        for (int w = 0; w < kWaves; ++w) wcount[w][t] = 0;
        __syncthreads();
        const long i = tile + (long)r * kBlock + t;
        const bool valid = i < n;
        uint64_t key = valid ? keys[i] : 0ull;
        uint32_t val = valid ? vals[i] : 0u;
        const uint32_t d = (uint32_t)(key >> shift) & 255u;
        // lanes of this wave holding the same digit
        unsigned long long m = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const unsigned long long bb = __ballot(bit);
            m &= bit ? bb : ~bb;
        }
        const uint32_t rank = (uint32_t)__popcll(m & lanes_below);
        if (valid && rank == 0) wcount[wave][d] = (uint32_t)__popcll(m);
        __syncthreads();
        uint32_t run = base[t];
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            woff[w][t] = run;
            run += wcount[w][t];
        }
        base[t] = run;
        __syncthreads();
        if (valid) {
            const uint32_t dst = woff[wave][d] + rank;
            keys_out[dst] = key;
            vals_out[dst] = val;
        }
        __syncthreads();
    }
}

inline int ceil_div(long a, long b) { return (int)((a + b - 1) / b); }

}  // namespace

size_t scan_temp_bytes(int n) { return sizeof(uint32_t) * (size_t)(ceil_div(n, kScanTile) + 1); }

void exclusive_scan_u32(const uint32_t* in, uint32_t* out, int n, void* temp, uint32_t* total_dev,
                        hipStream_t st)
{
    if (n <= 0) {
        if (total_dev) (void)hipMemsetAsync(total_dev, 0, sizeof(uint32_t), st);
        return;
    }
    const int nblk = ceil_div(n, kScanTile);
    uint32_t* sums = static_cast<uint32_t*>(temp);
    hipLaunchKernelGGL(k_scan_reduce, dim3(nblk), dim3(kBlock), 0, st, in, n, sums);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kBlock), 0, st, sums, nblk, total_dev);
    hipLaunchKernelGGL(k_scan_down, dim3(nblk), dim3(kBlock), 0, st, in, out, n, sums);
}

size_t radix_temp_bytes(int n)
{
    const int nblk = ceil_div(n > 0 ? n : 1, kSortTile);
    const size_t counts = (size_t)256 * nblk;
    return sizeof(uint32_t) * counts + scan_temp_bytes((int)counts) + 256;
}

void radix_sort_pairs(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt, uint32_t* vals_alt, int n,
                      int nbits, void* temp, hipStream_t st, bool* result_in_alt)
{
    *result_in_alt = false;
    if (n <= 1 || nbits <= 0) return;
    const int nblk = ceil_div(n, kSortTile);
    const int ncounts = 256 * nblk;
    uint32_t* counts = static_cast<uint32_t*>(temp);
    char* scan_tmp = reinterpret_cast<char*>(counts + ncounts);
    scan_tmp += (256 - (reinterpret_cast<uintptr_t>(scan_tmp) & 255)) & 255;
    uint64_t* kin = keys;
    uint32_t* vin = vals;
    uint64_t* kout = keys_alt;
    uint32_t* vout = vals_alt;
    for (int shift = 0; shift < nbits; shift += 8) {
        hipLaunchKernelGGL(k_radix_hist, dim3(nblk), dim3(kBlock), 0, st, kin, n, shift, counts, nblk);
        exclusive_scan_u32(counts, counts, ncounts, scan_tmp, nullptr, st);
        hipLaunchKernelGGL(k_radix_scatter, dim3(nblk), dim3(kBlock), 0, st, kin, vin, kout, vout, n, shift,
                           counts, nblk);
        std::swap(kin, kout);
        std::swap(vin, vout);
        *result_in_alt = !*result_in_alt;
    }
}

}  // namespace dem
