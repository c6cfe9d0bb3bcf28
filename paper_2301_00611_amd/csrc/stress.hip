// stress.hip -- reporting kernels: per-pair forces (read back by the
// contact list and the wall reactions) and the sums over the contact
// network: the Love-Weber stress, the normal springs' modulus of the
// stress-controlled cell and the mean contact force of the unbalanced force
// (utils.getStress, section 5 utility reference): the sum over the real
// sphere-sphere contacts of f (x) l, where f is the force on #2 and l the
// branch vector from #2 to #1, so that repulsive contacts give negative
// (compressive) stress.  Divided by the volume on the host.
//
// Run on demand, not in the step: it reads the pair records the last step
// wrote.  The branch is rebuilt from the stored normal and overlap:
// l = -(r1 + r2 - pen) n with pen = |F - Fs| / kn, the same quantities the
// contact kernel used.  One partial sum of 9 doubles per block, combined in
// a fixed order (waves, then blocks on the host): deterministic.
#include "dem_internal.hpp"

#include <algorithm>
#include <mutex>

namespace dem {

// The fixed device scratch of dem_get_stress_noalloc (see below): 1025 x 9
// doubles (73,800 bytes) on every GPU the library runs on, held until the
// process ends.
static __device__ __align__(256) double scratch[(1024 + 1) * 9];

namespace {

constexpr int kStressBlock = 256;

// Force on #2 of pair k (0 unless the pair touched at the last step): from
// its force record, or (FP64 linear law) its history record, fn n + Fs
// (without contraction, as the force sum forms it).
template <int PREC>
__device__ inline void pair_force(const StepArgs& a, int k, double* F)
{
#pragma clang fp contract(off)
    F[0] = F[1] = F[2] = 0.0;
    if (!a.pr.real[k]) return;
    if (!a.use_frec) {
        const HistRec h = hist_load<PREC>(a.pr.h, k);
        F[0] = h.fn * h.nx + h.fsx;
        F[1] = h.fn * h.ny + h.fsy;
        F[2] = h.fn * h.nz + h.fsz;
    } else if (PREC == DEM_FP32_MIXED) {
        const float* q = a.pr.frecf + (size_t)kForceWords * k;
        F[0] = q[0];
        F[1] = q[1];
        F[2] = q[2];
    } else {
        const double* q = a.pr.frec + (size_t)kForceWords * k;
        F[0] = q[0];
        F[1] = q[1];
        F[2] = q[2];
    }
}

// The largest overlap ratio over the touching pairs: wave maxima, then an
// integer maximum on the bits (non-negative doubles order like their bits).
template <int PREC>
__global__ void __launch_bounds__(kStressBlock) k_max_overlap(StepArgs a, unsigned long long* __restrict__ out)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    double v = 0.0;
    if (k < a.npairs && a.pr.real[k]) {
        const double pen = hist_load<PREC>(a.pr.h, k).pen;
        const int32_t sa = a.pr.a[k], sb = a.pr.b[k];
        const double r2 = a.bod.xr[sb].w;
        const double rmin = sa < 0 ? r2 : fmin(a.bod.xr[sa].w, r2);
        v = pen / rmin;
    }
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
    if ((threadIdx.x & 63) == 0 && v > 0.0) atomicMax(out, (unsigned long long)__double_as_longlong(v));
}

// Per-pair force on #2 (3 doubles per pair) for reporting.
template <int PREC>
__global__ void __launch_bounds__(kStressBlock) k_pair_forces(StepArgs a, double* __restrict__ f3)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.npairs) return;
    double F[3];
    pair_force<PREC>(a, k, F);
    f3[3 * (size_t)k + 0] = F[0];
    f3[3 * (size_t)k + 1] = F[1];
    f3[3 * (size_t)k + 2] = F[2];
}

// The terms of pair k for the sums over the real contacts of one scene
// (kNetworkWords doubles): the Love-Weber stress (9, sphere-sphere
// contacts), the normal springs' modulus k_n (d_i n_i)^2 per axis (3,
// sphere-sphere; d = (r1 + r2 - pen) n is the centre distance vector), |F|
// and 1 (walls included; unbalanced force).  Zero for a pair not touching.
template <int PREC, bool BATCHED>
__device__ inline void network_terms(const StepArgs& a, int k, int scene, double* s)
{
    for (int q = 0; q < kNetworkWords; ++q) s[q] = 0.0;
    const Pairs& P = a.pr;
    if (k >= a.npairs || !P.real[k]) return;
    const Bodies& B = a.bod;
    const int sa = P.a[k], sb = P.b[k];
    if (BATCHED && (int)B.scene[sb] != scene) return;
    double F[3];
    pair_force<PREC>(a, k, F);
    s[12] = sqrt(F[0] * F[0] + F[1] * F[1] + F[2] * F[2]);
    s[13] = 1.0;
    if (sa < 0) return;
    const HistRec h = hist_load<PREC>(P.h, k);
    const double n[3] = {h.nx, h.ny, h.nz};
    const double fn[3] = {F[0] - h.fsx, F[1] - h.fsy, F[2] - h.fsz};
    const double r1 = B.xr[sa].w, r2 = B.xr[sb].w;
    const Material M1 = a.mats[B.mat[sa]], M2 = a.mats[B.mat[sb]];
    const double k1 = M1.young * (2.0 * r1), k2 = M2.young * (2.0 * r2);
    const double kn = k1 * k2 / (k1 + k2);
    const double pen = sqrt(fn[0] * fn[0] + fn[1] * fn[1] + fn[2] * fn[2]) / kn;
    const double lm = (r1 + r2) - pen;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) s[3 * i + j] = F[i] * (-lm * n[j]);
    for (int i = 0; i < 3; ++i) {
        const double dn = (lm * n[i]) * n[i];
        s[9 + i] = kn * dn * dn;
    }
}

// Block sum of kNetworkWords terms in a fixed order (waves, then the
// block's waves in order), written to part[blockIdx.x].
__device__ inline void block_store_terms(double* s, double* __restrict__ part)
{
    __shared__ double sh[kStressBlock / 64][kNetworkWords];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int q = 0; q < kNetworkWords; ++q)
        for (int off = 32; off > 0; off >>= 1) s[q] += __shfl_down(s[q], off, 64);
    if (lane == 0)
        for (int q = 0; q < kNetworkWords; ++q) sh[wave][q] = s[q];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int q = 0; q < kNetworkWords; ++q) {
            double t = 0.0;
            for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[w][q];
            part[kNetworkWords * (size_t)blockIdx.x + q] = t;
        }
}

// On demand (reports): one scene's sums, one partial per block.
template <int PREC, bool BATCHED>
__global__ void __launch_bounds__(kStressBlock) k_network(StepArgs a, int scene, double* __restrict__ part)
{
    double s[kNetworkWords];
    network_terms<PREC, BATCHED>(a, blockIdx.x * blockDim.x + threadIdx.x, scene, s);
    block_store_terms(s, part);
}

constexpr int kNoAllocBlocks = 1024;
constexpr int kNoAllocWords = 9;

// ---- the Love-Weber stress without any allocation (dem_get_stress_noalloc)
//
// Its partial sums live in `scratch`, a fixed device array of this file: at
// most kNoAllocBlocks blocks, each striding over the pairs (thread t of block
// b takes pairs b B + t + j G B, j = 0, 1, ..., in that order), store their
// nine sums, and one more block adds the blocks' sums in block order into
// the array's last nine words.  Every word read is written first by the same
// call, so nothing needs clearing; two calls that overlap on one GPU share
// the array and race.

template <int PREC, bool BATCHED>
__global__ void __launch_bounds__(kStressBlock) k_stress_strided(StepArgs a, int scene, int per_thread,
                                                                  double* __restrict__ part)
{
    double acc[kNetworkWords];
    for (int q = 0; q < kNetworkWords; ++q) acc[q] = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int j = 0; j < per_thread; ++j, k += stride) {
        if (k >= a.npairs) break;
        double t[kNetworkWords];
        network_terms<PREC, BATCHED>(a, (int)k, scene, t);
        for (int q = 0; q < kNoAllocWords; ++q) acc[q] += t[q];
    }
    // the block's sums of the nine stress words, waves in order
    __shared__ double sh[kStressBlock / 64][kNoAllocWords];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int q = 0; q < kNoAllocWords; ++q)
        for (int off = 32; off > 0; off >>= 1) acc[q] += __shfl_down(acc[q], off, 64);
    if (lane == 0)
        for (int q = 0; q < kNoAllocWords; ++q) sh[wave][q] = acc[q];
    __syncthreads();
    if (threadIdx.x < kNoAllocWords) {
        double v = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) v += sh[w][threadIdx.x];
        part[kNoAllocWords * (size_t)blockIdx.x + threadIdx.x] = v;
    }
}

// One block: word q of the total is the blocks' word q added in block order.
__global__ void __launch_bounds__(64) k_stress_final(const double* __restrict__ part, int nblocks,
                                                     double* __restrict__ out)
{
    if (threadIdx.x >= kNoAllocWords) return;
    double v = 0.0;
    for (int b = 0; b < nblocks; ++b) v += part[kNoAllocWords * (size_t)b + threadIdx.x];
    out[threadIdx.x] = v;
}

}  // namespace

// Device address of `scratch` on the current device, looked up once per
// device (each GPU holds its own copy of the array at its own address; the
// array's name in host code is only a stand-in for it).
static double* noalloc_scratch()
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static double* ptr[kMaxDevices] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
        ptr[dev] = static_cast<double*>(p);
    }
    return ptr[dev];
}

int64_t stress_noalloc_max_pairs() { return (int64_t)kNoAllocBlocks * kStressBlock * kNoAllocMaxPerThread; }

const double* launch_stress_noalloc(const StepArgs& a, int precision, bool batched, int scene, hipStream_t st)
{
    double* base = noalloc_scratch();
    if (!base) return nullptr;
    if (a.npairs <= 0 || (int64_t)a.npairs > stress_noalloc_max_pairs()) return nullptr;
    const int grid = std::min(stress_blocks(a.npairs), kNoAllocBlocks);
    const int64_t span = (int64_t)grid * kStressBlock;
    const int per_thread = (int)((a.npairs + span - 1) / span);
    static_assert(sizeof(scratch) == sizeof(double) * (kNoAllocBlocks + 1) * kNoAllocWords, "scratch size");
    double* out = base + (size_t)kNoAllocBlocks * kNoAllocWords;
    if (precision == DEM_FP32_MIXED) {
        if (batched)
            hipLaunchKernelGGL((k_stress_strided<DEM_FP32_MIXED, true>), dim3(grid), dim3(kStressBlock), 0, st, a, scene,
                               per_thread, base);
        else
            hipLaunchKernelGGL((k_stress_strided<DEM_FP32_MIXED, false>), dim3(grid), dim3(kStressBlock), 0, st, a,
                               scene, per_thread, base);
    } else {
        if (batched)
            hipLaunchKernelGGL((k_stress_strided<DEM_FP64, true>), dim3(grid), dim3(kStressBlock), 0, st, a, scene,
                               per_thread, base);
        else
            hipLaunchKernelGGL((k_stress_strided<DEM_FP64, false>), dim3(grid), dim3(kStressBlock), 0, st, a, scene,
                               per_thread, base);
    }
    hipLaunchKernelGGL(k_stress_final, dim3(1), dim3(64), 0, st, (const double*)base, grid, out);
    return out;
}

void launch_pair_forces(const StepArgs& a, int precision, double* f3, hipStream_t st)
{
    const int grid = stress_blocks(a.npairs);
    if (grid == 0) return;
    if (precision == DEM_FP32_MIXED)
        hipLaunchKernelGGL(k_pair_forces<DEM_FP32_MIXED>, dim3(grid), dim3(kStressBlock), 0, st, a, f3);
    else
        hipLaunchKernelGGL(k_pair_forces<DEM_FP64>, dim3(grid), dim3(kStressBlock), 0, st, a, f3);
}

int stress_blocks(int npairs) { return npairs > 0 ? (npairs + kStressBlock - 1) / kStressBlock : 0; }

void launch_max_overlap(const StepArgs& a, int precision, unsigned long long* out, hipStream_t st)
{
    const int grid = stress_blocks(a.npairs);
    if (grid == 0) return;
    if (precision == DEM_FP32_MIXED)
        hipLaunchKernelGGL(k_max_overlap<DEM_FP32_MIXED>, dim3(grid), dim3(kStressBlock), 0, st, a, out);
    else
        hipLaunchKernelGGL(k_max_overlap<DEM_FP64>, dim3(grid), dim3(kStressBlock), 0, st, a, out);
}

void launch_network(const StepArgs& a, int precision, bool batched, int scene, double* part, hipStream_t st)
{
    const int grid = stress_blocks(a.npairs);
    if (grid == 0) return;
    if (precision == DEM_FP32_MIXED) {
        if (batched) hipLaunchKernelGGL((k_network<DEM_FP32_MIXED, true>), dim3(grid), dim3(kStressBlock), 0, st, a, scene, part);
        else hipLaunchKernelGGL((k_network<DEM_FP32_MIXED, false>), dim3(grid), dim3(kStressBlock), 0, st, a, scene, part);
    } else {
        if (batched) hipLaunchKernelGGL((k_network<DEM_FP64, true>), dim3(grid), dim3(kStressBlock), 0, st, a, scene, part);
        else hipLaunchKernelGGL((k_network<DEM_FP64, false>), dim3(grid), dim3(kStressBlock), 0, st, a, scene, part);
    }
}

}  // namespace dem
