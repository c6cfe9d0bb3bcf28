// broadphase.hip -- the collider's role (section 2.1.1, InsertionSortCollider)
// rebuilt for the GPU: bodies are binned in cells no smaller than the largest
// candidate distance (2 r_max + 2 Delta L), sorted by the Morton code of their
// cell, and each body sweeps the 27 cells around its own for candidates whose
// enlarged spheres overlap (distance < r_i + r_j + 2 Delta L).  The run is
// needed only when some body may have moved farther than Delta L since the
// last one (eq. 2.3-2.4).  Candidate pairs are stored once (owner = #1 of the
// contact); every body keeps a row of its candidate pairs sorted by partner
// id, and the shear history of surviving pairs is carried over by id.
#include "dem_internal.hpp"

#include <cfloat>

namespace dem {

namespace {

constexpr int kBlock = 256;
constexpr uint32_t kEmpty = 0xffffffffu;

__device__ inline uint64_t spread3(uint64_t v)
{
    v &= 0x1fffffull;
    v = (v | (v << 32)) & 0x1f00000000ffffull;
    v = (v | (v << 16)) & 0x1f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

__device__ inline uint32_t compact3(uint64_t v)
{
    v &= 0x1249249249249249ull;
    v = (v ^ (v >> 2)) & 0x10c30c30c30c30c3ull;
    v = (v ^ (v >> 4)) & 0x100f00f00f00f00full;
    v = (v ^ (v >> 8)) & 0x1f0000ff0000ffull;
    v = (v ^ (v >> 16)) & 0x1f00000000ffffull;
    v = (v ^ (v >> 32)) & 0x1fffffull;
    return (uint32_t)v;
}

__device__ inline uint64_t morton3(int x, int y, int z)
{
    return spread3((uint64_t)x) | (spread3((uint64_t)y) << 1) | (spread3((uint64_t)z) << 2);
}

__device__ inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Pack an integer image shift (each component in [-512, 511]) so that
// unsigned comparison orders shifts lexicographically.
__device__ inline int32_t pack_cell(int cx, int cy, int cz)
{
    return (int32_t)(((uint32_t)(cx + 512) << 20) | ((uint32_t)(cy + 512) << 10) | (uint32_t)(cz + 512));
}
__device__ inline void unpack_cell(int32_t p, int* c)
{
    uint32_t u = (uint32_t)p;
    c[0] = (int)((u >> 20) & 1023u) - 512;
    c[1] = (int)((u >> 10) & 1023u) - 512;
    c[2] = (int)(u & 1023u) - 512;
}
// packed (0, 0, 0): the shift of every aperiodic pair and every wall pair
constexpr int32_t kCellZero = (int32_t)((512u << 20) | (512u << 10) | 512u);
__device__ inline int32_t neg_cell(int32_t p)
{
    int c[3];
    unpack_cell(p, c);
    return pack_cell(-c[0], -c[1], -c[2]);
}

// One level of a scene's grid (level 1 exists only when r_split > 0).
struct Level {
    const double* origin;
    const double* inv_h;
    const double* cellw;
    const int32_t* dims;
    int32_t offset;
};
__device__ inline Level level_of(const SceneParams& P, int lv)
{
    return lv == 0 ? Level{P.origin, P.inv_h, P.cellw, P.dims, P.cell_offset}
                   : Level{P.origin2, P.inv_h2, P.cellw2, P.dims2, P.cell_offset2};
}
// the level a sphere of radius r is binned on
__device__ inline int level_of_radius(const SceneParams& P, double r) { return (P.r_split > 0.0 && r > P.r_split) ? 1 : 0; }

// Cell of a body on one level and, in a periodic cell, its integer period.
template <bool PERIODIC>
__device__ inline void cell_of(const SceneParams& P, const Level& V, double x, double y, double z, int* c, int* per)
{
    if (!PERIODIC) {
        c[0] = clampi((int)floor((x - V.origin[0]) * V.inv_h[0]), 0, V.dims[0] - 1);
        c[1] = clampi((int)floor((y - V.origin[1]) * V.inv_h[1]), 0, V.dims[1] - 1);
        c[2] = clampi((int)floor((z - V.origin[2]) * V.inv_h[2]), 0, V.dims[2] - 1);
        per[0] = per[1] = per[2] = 0;
        return;
    }
    const double* M = P.Hinv;
    double f[3] = {M[0] * x + M[1] * y + M[2] * z, M[3] * x + M[4] * y + M[5] * z, M[6] * x + M[7] * y + M[8] * z};
    for (int k = 0; k < 3; ++k) {
        double p = floor(f[k]);
        per[k] = (int)p;
        c[k] = clampi((int)floor((f[k] - p) * V.inv_h[k]), 0, V.dims[k] - 1);
    }
}

__device__ inline unsigned long long ord_bits(double v)
{
    unsigned long long b = (unsigned long long)__double_as_longlong(v);
    return (b & 0x8000000000000000ull) ? ~b : (b | 0x8000000000000000ull);
}

// ------------------------------------------------------------------ bounds

__global__ void __launch_bounds__(kBlock) k_bounds(Bodies b, int nslots, int batched,
                                                   unsigned long long* __restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < nslots;
    const int s = valid && batched ? (int)b.scene[i] : 0;
    unsigned long long v[6];
    if (valid) {
        const double4 p = b.xr[i];
        v[0] = ~ord_bits(p.x);
        v[1] = ~ord_bits(p.y);
        v[2] = ~ord_bits(p.z);
        v[3] = ord_bits(p.x);
        v[4] = ord_bits(p.y);
        v[5] = ord_bits(p.z);
    } else {
        for (int k = 0; k < 6; ++k) v[k] = 0ull;
    }
    // every value is reduced as a maximum (minima are stored complemented)
    const int s0 = __shfl(s, 0, 64);
    const bool uniform = __all(!valid || s == s0);
    if (uniform) {
        for (int k = 0; k < 6; ++k)
            for (int off = 32; off > 0; off >>= 1) {
                unsigned long long o = __shfl_xor(v[k], off, 64);
                v[k] = o > v[k] ? o : v[k];
            }
        if ((threadIdx.x & 63) == 0 && __any(valid))
            for (int k = 0; k < 6; ++k) atomicMax(&out[s0 * 6 + k], v[k]);
    } else if (valid) {
        for (int k = 0; k < 6; ++k) atomicMax(&out[s * 6 + k], v[k]);
    }
}

// Single scene: block maxima of the six ordered values, then one block
// combines them (no contended atomics).
__global__ void __launch_bounds__(kBlock) k_bounds_block(Bodies b, int nslots, unsigned long long* __restrict__ part)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long v[6] = {0ull, 0ull, 0ull, 0ull, 0ull, 0ull};
    if (i < nslots) {
        const double4 p = b.xr[i];
        v[0] = ~ord_bits(p.x);
        v[1] = ~ord_bits(p.y);
        v[2] = ~ord_bits(p.z);
        v[3] = ord_bits(p.x);
        v[4] = ord_bits(p.y);
        v[5] = ord_bits(p.z);
    }
    for (int k = 0; k < 6; ++k)
        for (int off = 32; off > 0; off >>= 1) {
            const unsigned long long o = __shfl_xor(v[k], off, 64);
            v[k] = o > v[k] ? o : v[k];
        }
    __shared__ unsigned long long s[kBlock / 64][6];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
        for (int k = 0; k < 6; ++k) s[wave][k] = v[k];
    __syncthreads();
    if (threadIdx.x < 6) {
        unsigned long long m = 0ull;
        for (int w = 0; w < kBlock / 64; ++w) m = s[w][threadIdx.x] > m ? s[w][threadIdx.x] : m;
        part[(long)blockIdx.x * 6 + threadIdx.x] = m;
    }
}

__global__ void __launch_bounds__(kBlock) k_bounds_final(const unsigned long long* __restrict__ part, int nblk,
                                                         unsigned long long* __restrict__ out)
{
    unsigned long long v[6] = {0ull, 0ull, 0ull, 0ull, 0ull, 0ull};
    for (int b = threadIdx.x; b < nblk; b += blockDim.x)
        for (int k = 0; k < 6; ++k) {
            const unsigned long long o = part[(long)b * 6 + k];
            v[k] = o > v[k] ? o : v[k];
        }
    for (int k = 0; k < 6; ++k)
        for (int off = 32; off > 0; off >>= 1) {
            const unsigned long long o = __shfl_xor(v[k], off, 64);
            v[k] = o > v[k] ? o : v[k];
        }
    __shared__ unsigned long long s[kBlock / 64][6];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
        for (int k = 0; k < 6; ++k) s[wave][k] = v[k];
    __syncthreads();
    if (threadIdx.x < 6) {
        unsigned long long m = 0ull;
        for (int w = 0; w < kBlock / 64; ++w) m = s[w][threadIdx.x] > m ? s[w][threadIdx.x] : m;
        out[threadIdx.x] = m;
    }
}

__global__ void k_bounds_decode(unsigned long long* __restrict__ bits, double* __restrict__ out, int n6)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n6) return;
    unsigned long long v = bits[i];
    if (i % 6 < 3) v = ~v;
    unsigned long long raw = (v & 0x8000000000000000ull) ? (v & 0x7fffffffffffffffull) : ~v;
    out[i] = __longlong_as_double((long long)raw);
}

// -------------------------------------------------------------------- keys

template <bool BATCHED, bool PERIODIC>
__global__ void __launch_bounds__(kBlock) k_keys(GridArgs g, uint64_t* __restrict__ keys,
                                                 uint32_t* __restrict__ vals)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.nslots) return;
    const int s = BATCHED ? (int)g.bod.scene[i] : 0;
    const SceneParams& P = (BATCHED || PERIODIC) ? g.scenes[s] : g.scene0;
    int c[3], per[3];
    const double4 p = g.bod.xr[i];
    cell_of<PERIODIC>(P, level_of(P, 0), p.x, p.y, p.z, c, per);
    // key: scene | Morton code of the level-0 cell (every sphere)
    uint64_t key = morton3(c[0], c[1], c[2]);
    if (BATCHED) key |= (uint64_t)s << (3 * g.morton_bits);
    keys[i] = key;
    vals[i] = (uint32_t)i;
    if (PERIODIC) {
        // a period is packed in 10 bits per axis: farther than 512 periods
        // from the origin it would wrap, so the run is refused instead
        bool out = false;
        for (int k = 0; k < 3; ++k) out = out || per[k] < -512 || per[k] > 511;
        if (out) *g.period_range = 1;
        g.bod.period[i] = pack_cell(per[0], per[1], per[2]);
    }
}

// ----------------------------------------------------------------- permute

__global__ void __launch_bounds__(kBlock) k_permute(Bodies src, Bodies dst, const uint32_t* __restrict__ order,
                                                    int nslots, int batched, int periodic,
                                                    int32_t* __restrict__ slot_of_id)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nslots) return;
    const uint32_t o = order[i];
    dst.xr[i] = src.xr[o];
    const double4 v = src.vm[o];
    dst.vm[i] = make_double4(v.x, v.y, v.z, 0.0);  // a fresh Verlet account after every broad-phase run
    dst.w[i] = src.w[o];
    dst.q[i] = src.q[o];
    dst.mat[i] = src.mat[o];
    dst.blocked[i] = src.blocked[o];
    const int32_t id = src.id[o];
    dst.id[i] = id;
    if (batched) dst.scene[i] = src.scene[o];
    if (periodic) dst.period[i] = src.period[o];
    slot_of_id[id] = i;
}

// ------------------------------------------------------------------- cells

template <int LV>
__device__ inline int cell_linear(const GridArgs& g, uint64_t key)
{
    const uint64_t mmask = (3 * g.morton_bits >= 64) ? ~0ull : ((1ull << (3 * g.morton_bits)) - 1ull);
    const int s = g.nscenes > 1 ? (int)(key >> (3 * g.morton_bits)) : 0;
    const SceneParams& P = g.nscenes > 1 ? g.scenes[s] : g.scene0;
    const Level V = level_of(P, LV);
    const uint64_t m = key & mmask;
    const int cx = (int)compact3(m), cy = (int)compact3(m >> 1), cz = (int)compact3(m >> 2);
    return V.offset + cx + V.dims[0] * (cy + V.dims[1] * cz);
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t v, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void __launch_bounds__(kBlock) k_cells(GridArgs g, const uint64_t* __restrict__ keys,
                                                  uint32_t* __restrict__ cell_start, uint32_t* __restrict__ cell_end,
                                                  int ncells)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.nslots) return;
    const uint64_t k = keys[i];
    const int lin = cell_linear<0>(g, k);
    if (lin < 0 || lin >= ncells) return;
    if (i == 0 || keys[i - 1] != k) cell_start[lin] = (uint32_t)i;
    if (i == g.nslots - 1 || keys[i + 1] != k) cell_end[lin] = (uint32_t)(i + 1);
}

// ---------------------------------------------------- level 1 (two levels)

// flag[i] = 1 for a sphere above its scene's r_split
template <bool BATCHED>
__global__ void __launch_bounds__(kBlock) k_large_flags(GridArgs g, uint32_t* __restrict__ flag)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.nslots) return;
    const int s = BATCHED ? (int)g.bod.scene[i] : 0;
    const SceneParams& P = BATCHED ? g.scenes[s] : g.scene0;
    flag[i] = level_of_radius(P, g.bod.xr[i].w) == 1 ? 1u : 0u;
}

// the coarse-cell key and slot of each large sphere, at its scanned position
template <bool BATCHED, bool PERIODIC>
__global__ void __launch_bounds__(kBlock) k_large_keys(GridArgs g, const uint32_t* __restrict__ scan,
                                                       uint64_t* __restrict__ keys2, uint32_t* __restrict__ vals2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.nslots) return;
    const uint32_t q = scan[i];
    if (scan[i + 1] == q) return;  // not a large sphere
    const int s = BATCHED ? (int)g.bod.scene[i] : 0;
    const SceneParams& P = (BATCHED || PERIODIC) ? g.scenes[s] : g.scene0;
    const double4 p = g.bod.xr[i];
    int c[3], per[3];
    cell_of<PERIODIC>(P, level_of(P, 1), p.x, p.y, p.z, c, per);
    uint64_t key = morton3(c[0], c[1], c[2]);
    if (BATCHED) key |= (uint64_t)s << (3 * g.morton_bits);
    keys2[q] = key;
    vals2[q] = (uint32_t)i;
}

__global__ void __launch_bounds__(kBlock) k_cells_large(GridArgs g, const uint64_t* __restrict__ keys2, int n,
                                                        uint32_t* __restrict__ cell_start,
                                                        uint32_t* __restrict__ cell_end, int ncells)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const uint64_t k = keys2[q];
    const int lin = cell_linear<1>(g, k);
    if (lin < 0 || lin >= ncells) return;
    if (q == 0 || keys2[q - 1] != k) cell_start[lin] = (uint32_t)q;
    if (q == n - 1 || keys2[q + 1] != k) cell_end[lin] = (uint32_t)(q + 1);
}

// ------------------------------------------------------------------- sweep

// A neighbour cell's index along one axis, wrapped into [0, dim) with the
// period crossed in w; outside an aperiodic grid the cell does not exist.
template <bool PERIODIC>
__device__ inline void wrap_axis(int& n, int dim, int& w, bool& skip)
{
    if (n < 0) {
        if (!PERIODIC) skip = true;
        n += dim;
        w = -1;
    } else if (n >= dim) {
        if (!PERIODIC) skip = true;
        n -= dim;
        w = 1;
    }
}

// Visit every candidate of home slot i (27 cells, then the scene's walls).
// f(partner_slot_or_wall, partner_id, packed_cell) is called per candidate.
// With SPLIT, the 64 lanes of a wave share one sphere's search: lane `part`
// visits every 64th group of cells, and every 64th wall.
template <bool BATCHED, bool PERIODIC, bool SPLIT = false, typename F>
__device__ inline void for_each_candidate(const SweepArgs& a, int i, F&& f, int part = 0)
{
    const GridArgs& g = a.g;
    const Bodies& B = g.bod;
    const int s = BATCHED ? (int)B.scene[i] : 0;
    const SceneParams& P = (BATCHED || PERIODIC) ? g.scenes[s] : g.scene0;
    const double4 pi = B.xr[i];
    const double xi = pi.x, yi = pi.y, zi = pi.z, ri = pi.w;
    const int32_t myid = B.id[i];
    const double reach = 2.0 * P.verlet;
    // level 0 holds every sphere; with two levels a sphere takes its
    // partners up to r_split there and the larger ones from level 1
    const bool two = P.r_split > 0.0;
    const int nlev = two ? 2 : 1;
    for (int lv = 0; lv < nlev; ++lv) {
    const Level V = level_of(P, lv);
    int c[3], per_i[3];
    cell_of<PERIODIC>(P, V, xi, yi, zi, c, per_i);
    // cells of this level within reach of this body's largest possible
    // candidate distance on it (the largest radius it takes there)
    const double far = (ri + (lv == 0 && two ? P.r_split : P.rmax)) + reach;
    int kk[3];
    for (int q = 0; q < 3; ++q) kk[q] = max(1, (int)ceil(far / V.cellw[q]));
    // test one sphere j (position and radius pj, packed period perj, id idj)
    // found across the periods (w0, w1, w2) of the home cell's neighbourhood
    auto visit = [&](uint32_t j, const double4& pj, int32_t perj_packed, int32_t idj, int w0, int w1, int w2) {
        if ((int)j == i) return;
        const double rj = pj.w;
        if (lv == 0 && two && rj > P.r_split) return;  // found on level 1
        const double sc = (ri + rj) + reach;
        double ddx, ddy, ddz;
        int32_t packed = kCellZero;
        if (PERIODIC) {
            int perj[3];
            unpack_cell(perj_packed, perj);
            const int cc[3] = {per_i[0] - perj[0] + w0, per_i[1] - perj[1] + w1, per_i[2] - perj[2] + w2};
            packed = pack_cell(cc[0], cc[1], cc[2]);
            // evaluate from the lower id's side so that both bodies of
            // a pair take the same decision
            const bool from_i = myid < idj;
            const int sg = from_i ? 1 : -1;
            const double* H = P.H;
            const double sx = (H[0] * (sg * cc[0]) + H[1] * (sg * cc[1])) + H[2] * (sg * cc[2]);
            const double sy = (H[3] * (sg * cc[0]) + H[4] * (sg * cc[1])) + H[5] * (sg * cc[2]);
            const double sz = (H[6] * (sg * cc[0]) + H[7] * (sg * cc[1])) + H[8] * (sg * cc[2]);
            const double ax = from_i ? xi : pj.x, ay = from_i ? yi : pj.y, az = from_i ? zi : pj.z;
            const double bx = from_i ? pj.x : xi, by = from_i ? pj.y : yi, bz = from_i ? pj.z : zi;
            ddx = (bx + sx) - ax;
            ddy = (by + sy) - ay;
            ddz = (bz + sz) - az;
        } else {
            ddx = pj.x - xi;
            ddy = pj.y - yi;
            ddz = pj.z - zi;
        }
        const double dd = (ddx * ddx + ddy * ddy) + ddz * ddz;
        if (dd < sc * sc) f((int32_t)j, idj, packed);
    };
    // one group of cells: up to three along x from (dx0, dy, dz); their
    // ranges are loaded together, then their spheres are visited as one
    // sequence, two at a time (the loads of both are issued before either
    // is tested)
    auto group = [&](int dz, int dy, int dx0) {
        int ny = c[1] + dy, nz = c[2] + dz, wy = 0, wz = 0;
        bool skip_row = false;
        wrap_axis<PERIODIC>(ny, V.dims[1], wy, skip_row);
        wrap_axis<PERIODIC>(nz, V.dims[2], wz, skip_row);
        if (skip_row) return;
        const int row_lin = V.offset + V.dims[0] * (ny + V.dims[1] * nz);
        uint32_t st[3], en[3];
        int wx[3];
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            int nx = c[0] + dx0 + t;
            bool skip = dx0 + t > kk[0];
            wx[t] = 0;
            wrap_axis<PERIODIC>(nx, V.dims[0], wx[t], skip);
            st[t] = kEmpty;
            en[t] = 0;
            if (!skip) {
                st[t] = a.cell_start[row_lin + nx];
                en[t] = a.cell_end[row_lin + nx];
            }
        }
        const uint32_t c0 = st[0] == kEmpty ? 0u : en[0] - st[0];
        const uint32_t c1 = st[1] == kEmpty ? 0u : en[1] - st[1];
        const uint32_t c2 = st[2] == kEmpty ? 0u : en[2] - st[2];
        const uint32_t tot = c0 + c1 + c2;
        auto at = [&](uint32_t k, int& wk) -> uint32_t {
            uint32_t q;
            if (k < c0) {
                q = st[0] + k;
                wk = wx[0];
            } else if (k < c0 + c1) {
                q = st[1] + (k - c0);
                wk = wx[1];
            } else {
                q = st[2] + (k - c0 - c1);
                wk = wx[2];
            }
            return lv == 0 ? q : g.large_slot[q];
        };
        for (uint32_t k = 0; k < tot; k += 2) {
            const bool two_here = k + 1 < tot;
            int wa, wb;
            const uint32_t ja = at(k, wa);
            const uint32_t jb = at(two_here ? k + 1 : k, wb);
            const double4 pa = B.xr[ja], pb = B.xr[jb];
            const int32_t pera = PERIODIC ? B.period[ja] : 0, perb = PERIODIC ? B.period[jb] : 0;
            const int32_t ida = B.id[ja], idb = B.id[jb];
            visit(ja, pa, pera, ida, wa, wy, wz);
            if (two_here) visit(jb, pb, perb, idb, wb, wy, wz);
        }
    };
    if (SPLIT) {
        // group gi = ((dz * ndy) + dy) * nch + chunk, lane `part` taking
        // every 64th, so that the wave's lanes search at the same time
        const int nch = (2 * kk[0] + 3) / 3, ndy = 2 * kk[1] + 1, ng = nch * ndy * (2 * kk[2] + 1);
        for (int gi = part; gi < ng; gi += 64) {
            const int ch = gi % nch, r = gi / nch;
            group(r / ndy - kk[2], r % ndy - kk[1], 3 * ch - kk[0]);
        }
    } else {
        for (int dz = -kk[2]; dz <= kk[2]; ++dz)
            for (int dy = -kk[1]; dy <= kk[1]; ++dy)
                for (int dx0 = -kk[0]; dx0 <= kk[0]; dx0 += 3) group(dz, dy, dx0);
    }
    }
    for (int k = SPLIT ? part : 0; k < P.wall_count; k += SPLIT ? 64 : 1) {
        const int wi = P.wall_begin + k;
        const Wall W = a.walls[wi];
        if (W.kind == kPlane) {
            const double xa = W.axis == 0 ? xi : (W.axis == 1 ? yi : zi);
            const double delta = xa - W.pos;
            if (fabs(delta) < ri + reach) f(-1 - wi, W.id, kCellZero);
        } else {
            // box or facet: closer than r + 2 Delta L to the primitive
            const double x[3] = {xi, yi, zi};
            if (boundary_distance(W, x) < ri + reach) f(-1 - wi, W.id, kCellZero);
        }
    }
}

// The sweeps run in two passes when a scene has two levels: the spheres of
// level 0 first, one per lane (a large sphere's lane returns at once), then
// the large ones through their index array, one per wave (a large sphere
// searches many more cells, which the wave's lanes share).
template <bool BATCHED>
__device__ inline int sweep_body(const SweepArgs& a)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.g.nslots) return -1;
    if (a.nlarge > 0) {
        const int s = BATCHED ? (int)a.g.bod.scene[t] : 0;
        const SceneParams& P = BATCHED ? a.g.scenes[s] : a.g.scene0;
        if (level_of_radius(P, a.g.bod.xr[t].w) == 1) return -1;
    }
    return t;
}

template <bool BATCHED, bool PERIODIC>
__global__ void __launch_bounds__(kBlock) k_sweep_count(SweepArgs a)
{
    const int i = sweep_body<BATCHED>(a);
    if (i < 0) return;
    uint32_t n = 0;
    for_each_candidate<BATCHED, PERIODIC>(a, i, [&](int32_t, int32_t, int32_t) { ++n; });
    a.count[i] = n;
}

// The level-1 sphere of a wave (-1 past the last: the whole wave returns).
__device__ inline int large_sphere_of_wave(const SweepArgs& a)
{
    const int t = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    return t < a.nlarge ? (int)a.g.large_slot[t] : -1;
}

template <bool BATCHED, bool PERIODIC>
__global__ void __launch_bounds__(kBlock) k_sweep_count_large(SweepArgs a)
{
    const int i = large_sphere_of_wave(a);
    if (i < 0) return;
    const int lane = threadIdx.x & 63;
    uint32_t n = 0;
    for_each_candidate<BATCHED, PERIODIC, true>(a, i, [&](int32_t, int32_t, int32_t) { ++n; }, lane);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) n += __shfl_down(n, off, 64);
    if (lane == 0) a.count[i] = n;
}

// How each row was left by the fill, kept in `count` (the counts are spent
// once the rows are laid out): already sorted, in the order found (sorted by
// the rank pass), or a level-1 row in the order found (sorted by the wave
// rank pass).
constexpr uint32_t kRowSorted = 0, kRowFound = 1, kRowLarge = 2;

// LDS pool of the level-0 fill: 8 entries per sphere of the block on
// average (24 KB, so that the six blocks per CU its registers allow fit).
constexpr int kStageEntries = 8 * kBlock;

// (partner id, packed image as unsigned) as one unsigned key
__device__ inline uint64_t row_key(int32_t pid, int32_t cell)
{
    return ((uint64_t)((uint32_t)pid ^ 0x80000000u) << 32) | (uint32_t)cell;
}

// The level-0 fill.  The rows of a block's spheres are contiguous, and the
// block takes them, in slot order, into its LDS pool while they fit: such a
// sweep stores nothing to memory (a store inside its loop would hold every
// later load until the store is done), then ranks its row in LDS and writes
// it sorted.  A row beyond the pool is written in the order found and
// sorted by the rank pass.
template <bool BATCHED, bool PERIODIC>
__global__ void __launch_bounds__(kBlock) k_sweep_fill_staged(SweepArgs a)
{
    __shared__ int32_t s_slot[kStageEntries];
    __shared__ int32_t s_pid[kStageEntries];
    __shared__ int32_t s_cell[kStageEntries];
    __shared__ uint32_t s_wave[kBlock / 64];
    const int i = sweep_body<BATCHED>(a);
    int beg = 0, len = 0;
    if (i >= 0) {
        beg = a.row_start[i];
        len = a.row_start[i + 1] - beg;
    }
    // the block's exclusive scan of the row lengths, in slot order
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t inc = (uint32_t)len;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(inc, off, 64);
        if (lane >= off) inc += y;
    }
    if (lane == 63) s_wave[wave] = inc;
    __syncthreads();
    uint32_t base = 0;
    for (int w = 0; w < wave; ++w) base += s_wave[w];
    if (i < 0) return;
    const uint32_t off = base + inc - (uint32_t)len;
    const bool staged = off + (uint32_t)len <= (uint32_t)kStageEntries;
    int n = 0;
    for_each_candidate<BATCHED, PERIODIC>(a, i, [&](int32_t slot, int32_t pid, int32_t cell) {
        if (n < len) {
            if (staged) {
                s_slot[off + n] = slot;
                s_pid[off + n] = pid;
                s_cell[off + n] = cell;
            } else {
                a.raw_slot[beg + n] = slot;
                a.raw_pid[beg + n] = pid;
                a.raw_cell[beg + n] = cell;
            }
        }
        ++n;
    });
    for (int e = 0; e < len; ++e) a.ent_body[beg + e] = i;
    if (!staged) {
        a.count[i] = kRowFound;
        return;
    }
    a.count[i] = kRowSorted;
    const int32_t myid = a.g.bod.id[i];
    for (int e = 0; e < len; ++e) {
        const int32_t slot = s_slot[off + e], pid = s_pid[off + e], cell = s_cell[off + e];
        const uint64_t ke = row_key(pid, cell);
        int rank = 0;
        for (int f = 0; f < len; ++f) {
            const uint64_t kf = row_key(s_pid[off + f], s_cell[off + f]);
            rank += (kf < ke || (kf == ke && f < e)) ? 1 : 0;
        }
        const int dst = beg + rank;
        a.ent_slot[dst] = slot;
        a.ent_pid[dst] = pid;
        a.ent_cell[dst] = cell;
        a.ent_own[dst] = (slot < 0 || myid < pid) ? 1u : 0u;
    }
}

// The level-1 fill, one wave per sphere: each lane counts the candidates
// of its groups of cells, then writes them after those of the lanes before
// it (the row is sorted afterwards, so this order only has to be complete).
template <bool BATCHED, bool PERIODIC>
__global__ void __launch_bounds__(kBlock) k_sweep_fill_large(SweepArgs a)
{
    const int i = large_sphere_of_wave(a);
    if (i < 0) return;
    const int lane = threadIdx.x & 63;
    uint32_t mine = 0;
    for_each_candidate<BATCHED, PERIODIC, true>(a, i, [&](int32_t, int32_t, int32_t) { ++mine; }, lane);
    uint32_t inc = mine;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(inc, off, 64);
        if (lane >= off) inc += y;
    }
    const int beg = a.row_start[i];
    const int cap = a.row_start[i + 1] - beg;
    int n = (int)(inc - mine);
    for_each_candidate<BATCHED, PERIODIC, true>(a, i, [&](int32_t slot, int32_t pid, int32_t cell) {
        if (n < cap) {
            a.raw_slot[beg + n] = slot;
            a.raw_pid[beg + n] = pid;
            a.raw_cell[beg + n] = cell;
            a.ent_body[beg + n] = i;
        }
        ++n;
    }, lane);
    if (lane == 0) a.count[i] = kRowLarge;
}

// One thread per entry of a level-0 row that the fill left in the order
// found: its place in its row sorted by (partner id, image as unsigned; ties
// by the order found, which cannot happen for distinct candidates) is the
// number of the row's entries before it in that order.  This order fixes the
// order of the force sum.
__global__ void __launch_bounds__(kBlock) k_row_rank(SweepArgs a)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= a.nent) return;
    const int i = a.ent_body[e];
    if (a.count[i] != kRowFound) return;
    const int beg = a.row_start[i], end = a.row_start[i + 1];
    const int32_t pid = a.raw_pid[e];
    const uint32_t cell = (uint32_t)a.raw_cell[e];
    int rank = 0;
    for (int f = beg; f < end; ++f) {
        const int32_t pf = a.raw_pid[f];
        const uint32_t cf = (uint32_t)a.raw_cell[f];
        rank += (pf < pid || (pf == pid && (cf < cell || (cf == cell && f < e)))) ? 1 : 0;
    }
    const int dst = beg + rank;
    const int32_t slot = a.raw_slot[e];
    a.ent_slot[dst] = slot;
    a.ent_pid[dst] = pid;
    a.ent_cell[dst] = (int32_t)cell;
    a.ent_own[dst] = (slot < 0 || a.g.bod.id[i] < pid) ? 1u : 0u;
}

// One wave per level-1 sphere: its row, the longest kind, ranked as above
// with the row's keys in LDS (a row longer than the wave's share is ranked
// from memory).
constexpr int kLargeRowLds = 1024;

__global__ void __launch_bounds__(kBlock) k_row_rank_large(SweepArgs a)
{
    __shared__ uint64_t s_key[kBlock / 64][kLargeRowLds];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int t = blockIdx.x * (kBlock / 64) + wave;
    if (t >= a.nlarge) return;  // the whole wave
    const int i = (int)a.g.large_slot[t];
    const int beg = a.row_start[i], len = a.row_start[i + 1] - beg;
    const bool in_lds = len <= kLargeRowLds;
    if (in_lds) {
        for (int f = lane; f < len; f += 64) s_key[wave][f] = row_key(a.raw_pid[beg + f], a.raw_cell[beg + f]);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
    const int32_t myid = a.g.bod.id[i];
    for (int e = lane; e < len; e += 64) {
        const int32_t slot = a.raw_slot[beg + e], pid = a.raw_pid[beg + e], cell = a.raw_cell[beg + e];
        const uint64_t ke = row_key(pid, cell);
        int rank = 0;
        if (in_lds) {
            for (int f = 0; f < len; ++f) {
                const uint64_t kf = s_key[wave][f];
                rank += (kf < ke || (kf == ke && f < e)) ? 1 : 0;
            }
        } else {
            for (int f = 0; f < len; ++f) {
                const uint64_t kf = row_key(a.raw_pid[beg + f], a.raw_cell[beg + f]);
                rank += (kf < ke || (kf == ke && f < e)) ? 1 : 0;
            }
        }
        const int dst = beg + rank;
        a.ent_slot[dst] = slot;
        a.ent_pid[dst] = pid;
        a.ent_cell[dst] = cell;
        a.ent_own[dst] = (slot < 0 || myid < pid) ? 1u : 0u;
    }
}

// -------------------------------------------------------- pairs and history

// One thread per row entry: an owning entry writes its pair (canonical
// index = the scan of the owner flags) and its row entry; the other finds
// its pair by binary search in the partner's sorted row.  The first entry of
// a row also writes the body's range of owned pairs.
__global__ void __launch_bounds__(kBlock) k_pair_build(PairBuildArgs a)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= a.nent) return;
    const int i = a.ent_body[e];
    const int32_t myid = a.bod.id[i];
    const int32_t slot = a.ent_slot[e];
    if (a.ent_own[e]) {
        const uint32_t k = a.own_scan[e];
        if (slot < 0) {
            // a wall pair: the wall is #1 and has no row
            a.ca[k] = slot;
            a.cb[k] = i;
            a.rows.ent[e] = k;
        } else {
            a.ca[k] = i;
            a.cb[k] = slot;
            a.rows.ent[e] = k | kNegSign;
        }
        a.hist_new.cell[k] = a.ent_cell[e];
        a.hist_new.pid[k] = a.ent_pid[e];
    } else {
        // the pair is owned by the partner: find this body in its row,
        // which is sorted by (partner id, packed image as unsigned)
        const uint32_t want = (uint32_t)neg_cell(a.ent_cell[e]);
        int lo = a.row_start[slot], hi = a.row_start[slot + 1];
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            const int32_t pm = a.ent_pid[mid];
            const uint32_t cm = (uint32_t)a.ent_cell[mid];
            if (pm < myid || (pm == myid && cm < want))
                lo = mid + 1;
            else
                hi = mid;
        }
        uint32_t k = kPairMask;
        if (lo < a.row_start[slot + 1] && a.ent_pid[lo] == myid && (uint32_t)a.ent_cell[lo] == want &&
            a.ent_own[lo])
            k = a.own_scan[lo];
        a.rows.ent[e] = k;
    }
    const int beg = a.row_start[i];
    if (e == beg) {
        const int end = a.row_start[i + 1];
        a.hist_new.own_begin[myid] = (int32_t)a.own_scan[beg];
        a.hist_new.own_count[myid] = (int32_t)(a.own_scan[end] - a.own_scan[beg]);
    }
}

// Per canonical pair: where its history sits in the previous list, and
// whether that history says the pair touched (a carried normal is a unit
// vector; a new pair starts with zero shear force and no normal).
__global__ void __launch_bounds__(kBlock) k_carry_find(PairBuildArgs a, int old_nbodies)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > a.npairs) return;
    if (k == a.npairs) {
        a.flag[k] = 0u;  // the scan's extra entry
        return;
    }
    const int32_t sa = a.ca[k], sb = a.cb[k];
    const int32_t owner = sa >= 0 ? a.bod.id[sa] : a.bod.id[sb];
    const int32_t partner = a.hist_new.pid[k];
    const int32_t cell = a.hist_new.cell[k];
    int32_t found = -1;
    if (a.has_old && owner < old_nbodies) {
        const int lo = a.hist_old.own_begin[owner];
        const int cnt = a.hist_old.own_count[owner];
        for (int q = lo; q < lo + cnt; ++q) {
            if (a.hist_old.pid[q] == partner && a.hist_old.cell[q] == cell) {
                found = a.hist_old.map[q];
                break;
            }
        }
    }
    bool touched = false;
    if (found >= 0) {
        const HistRec h = a.hist_f32 ? widen(reinterpret_cast<const HistRec32*>(a.hist_old.h)[found])
                                     : a.hist_old.h[found];
        touched = h.nx != 0.0 || h.ny != 0.0 || h.nz != 0.0;
    }
    a.found[k] = found;
    a.flag[k] = touched ? 1u : 0u;
}

// The stable partition, within each eighth [P_x, P_x+1) of the pairs
// (P_x = x npairs / 8, the segment one XCD takes in the contact kernel) and
// within each chunk of kPartitionChunk pairs of it: touching pairs first,
// then the others, each group in canonical order; the history moves with its
// pair, and the canonical -> final map is kept for the next run.  Chunks keep
// a body's touching and non-touching pairs close in time in the contact
// kernel, so the positions the second group gathers are still cached.
__device__ inline uint32_t segment_start(int x, int npairs) { return (uint32_t)(((int64_t)x * npairs) >> 3); }
constexpr uint32_t kPartitionChunk = 1u << 14;

__global__ void __launch_bounds__(kBlock) k_partition(PairBuildArgs a)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.npairs) return;
    int x = (int)(((int64_t)k * 8) / a.npairs);
    if (x > 7) x = 7;
    while (x < 7 && (uint32_t)k >= segment_start(x + 1, a.npairs)) ++x;
    while (x > 0 && (uint32_t)k < segment_start(x, a.npairs)) --x;
    const uint32_t x0 = segment_start(x, a.npairs), x1 = segment_start(x + 1, a.npairs);
    const uint32_t p0 = x0 + (((uint32_t)k - x0) / kPartitionChunk) * kPartitionChunk;
    const uint32_t p1 = min(p0 + kPartitionChunk, x1);
    const uint32_t s0 = a.flag_scan[p0];
    const uint32_t ntouch = a.flag_scan[p1] - s0;
    const uint32_t r = a.flag_scan[k] - s0;
    const bool touched = a.flag[k] != 0u;
    const uint32_t pos = p0 + (touched ? r : ntouch + (((uint32_t)k - p0) - r));
    a.pr.a[pos] = a.ca[k];
    a.pr.b[pos] = a.cb[k];
    a.pr.cell[pos] = a.hist_new.cell[k];
    a.pr.pid[pos] = a.hist_new.pid[k];
    const int32_t f = a.found[k];
    if (a.hist_f32)
        reinterpret_cast<HistRec32*>(a.pr.h)[pos] =
            f >= 0 ? reinterpret_cast<const HistRec32*>(a.hist_old.h)[f] : HistRec32{};
    else
        a.pr.h[pos] = f >= 0 ? a.hist_old.h[f] : HistRec{};
    a.pr.real[pos] = touched ? 1 : 0;
    a.pr.ea[pos] = -1;  // set below from the rows (stays -1 for a boundary pair)
    a.pr.eb[pos] = -1;
    a.hist_new.map[k] = (int32_t)pos;
}

// Row entries: canonical pair index -> partitioned index (the side bit kept,
// the touched bit from the carried history); each pair learns where its
// entries sit, so that the contact kernel can update their touched bits.
__global__ void __launch_bounds__(kBlock) k_remap_rows(PairBuildArgs a)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= a.nent) return;
    const uint32_t u = a.rows.ent[e];
    const uint32_t k = u & kPairMask;
    if (k < (uint32_t)a.npairs) {
        const uint32_t pos = (uint32_t)a.hist_new.map[k];
        a.rows.ent[e] = (u & kNegSign) | (a.flag[k] ? kRealBit : 0u) | pos;
        if (u & kNegSign)
            a.pr.ea[pos] = e;
        else
            a.pr.eb[pos] = e;
    }
}

inline int nblocks(long n) { return (int)((n + kBlock - 1) / kBlock); }

}  // namespace

size_t bounds_temp_bytes(int nslots) { return sizeof(unsigned long long) * 6 * (size_t)(nblocks(nslots) + 1); }

void launch_bounds(const Bodies& b, int nslots, int nscenes, double* out6, void* temp, hipStream_t st)
{
    // out6 doubles as the buffer of ordered bits (same size)
    unsigned long long* bits = reinterpret_cast<unsigned long long*>(out6);
    (void)hipMemsetAsync(bits, 0, sizeof(unsigned long long) * 6 * nscenes, st);
    if (nslots > 0) {
        if (nscenes == 1) {
            unsigned long long* part = static_cast<unsigned long long*>(temp);
            hipLaunchKernelGGL(k_bounds_block, dim3(nblocks(nslots)), dim3(kBlock), 0, st, b, nslots, part);
            hipLaunchKernelGGL(k_bounds_final, dim3(1), dim3(kBlock), 0, st, part, nblocks(nslots), bits);
        } else {
            // bodies are grouped by scene after the first run, so nearly every
            // wave is uniform and the atomics spread over the scenes
            hipLaunchKernelGGL(k_bounds, dim3(nblocks(nslots)), dim3(kBlock), 0, st, b, nslots, 1, bits);
        }
    }
    hipLaunchKernelGGL(k_bounds_decode, dim3(nblocks(6 * nscenes)), dim3(kBlock), 0, st, bits, out6, 6 * nscenes);
}

void launch_keys(const GridArgs& g, uint64_t* keys, uint32_t* vals, hipStream_t st)
{
    if (g.nslots <= 0) return;
    const bool batched = g.nscenes > 1;
    const bool periodic = g.scene0.periodic != 0;
    dim3 grid(nblocks(g.nslots)), blk(kBlock);
    if (batched)
        hipLaunchKernelGGL((k_keys<true, false>), grid, blk, 0, st, g, keys, vals);
    else if (periodic)
        hipLaunchKernelGGL((k_keys<false, true>), grid, blk, 0, st, g, keys, vals);
    else
        hipLaunchKernelGGL((k_keys<false, false>), grid, blk, 0, st, g, keys, vals);
}

void launch_permute(const Bodies& src, const Bodies& dst, const uint32_t* order, int nslots, bool batched,
                    bool periodic, int32_t* slot_of_id, hipStream_t st)
{
    if (nslots <= 0) return;
    hipLaunchKernelGGL(k_permute, dim3(nblocks(nslots)), dim3(kBlock), 0, st, src, dst, order, nslots,
                       batched ? 1 : 0, periodic ? 1 : 0, slot_of_id);
}

void launch_cells(const GridArgs& g, const uint64_t* sorted_keys, uint32_t* cell_start, uint32_t* cell_end,
                  int ncells, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill_u32, dim3(nblocks(ncells)), dim3(kBlock), 0, st, cell_start, kEmpty, ncells);
    hipLaunchKernelGGL(k_fill_u32, dim3(nblocks(ncells)), dim3(kBlock), 0, st, cell_end, 0u, ncells);
    if (g.nslots > 0)
        hipLaunchKernelGGL(k_cells, dim3(nblocks(g.nslots)), dim3(kBlock), 0, st, g, sorted_keys, cell_start,
                           cell_end, ncells);
}

void launch_large_flags(const GridArgs& g, uint32_t* flag, hipStream_t st)
{
    if (g.nslots <= 0) return;
    if (g.nscenes > 1)
        hipLaunchKernelGGL((k_large_flags<true>), dim3(nblocks(g.nslots)), dim3(kBlock), 0, st, g, flag);
    else
        hipLaunchKernelGGL((k_large_flags<false>), dim3(nblocks(g.nslots)), dim3(kBlock), 0, st, g, flag);
}

void launch_large_keys(const GridArgs& g, const uint32_t* scan, uint64_t* keys2, uint32_t* vals2, hipStream_t st)
{
    if (g.nslots <= 0) return;
    dim3 grid(nblocks(g.nslots)), blk(kBlock);
    if (g.nscenes > 1)
        hipLaunchKernelGGL((k_large_keys<true, false>), grid, blk, 0, st, g, scan, keys2, vals2);
    else if (g.scene0.periodic)
        hipLaunchKernelGGL((k_large_keys<false, true>), grid, blk, 0, st, g, scan, keys2, vals2);
    else
        hipLaunchKernelGGL((k_large_keys<false, false>), grid, blk, 0, st, g, scan, keys2, vals2);
}

void launch_cells_large(const GridArgs& g, const uint64_t* sorted_keys2, int nlarge, uint32_t* cell_start,
                        uint32_t* cell_end, int ncells, hipStream_t st)
{
    if (nlarge > 0)
        hipLaunchKernelGGL(k_cells_large, dim3(nblocks(nlarge)), dim3(kBlock), 0, st, g, sorted_keys2, nlarge,
                           cell_start, cell_end, ncells);
}

// The level-0 pass (one sphere per lane) and, with two levels, the level-1
// pass (one sphere per wave) of a sweep kernel pair.
#define DEM_SWEEP_LAUNCH(SMALL, LARGE_K, A, ST)                                                                \
    do {                                                                                                      \
        const dim3 blk(kBlock), g0(nblocks((A).g.nslots));                                                    \
        const dim3 g1(((A).nlarge + kBlock / 64 - 1) / (kBlock / 64));                                        \
        if ((A).g.nscenes > 1) {                                                                              \
            hipLaunchKernelGGL((SMALL<true, false>), g0, blk, 0, ST, A);                                      \
            if ((A).nlarge > 0) hipLaunchKernelGGL((LARGE_K<true, false>), g1, blk, 0, ST, A);                \
        } else if ((A).g.scene0.periodic) {                                                                   \
            hipLaunchKernelGGL((SMALL<false, true>), g0, blk, 0, ST, A);                                      \
            if ((A).nlarge > 0) hipLaunchKernelGGL((LARGE_K<false, true>), g1, blk, 0, ST, A);                \
        } else {                                                                                              \
            hipLaunchKernelGGL((SMALL<false, false>), g0, blk, 0, ST, A);                                     \
            if ((A).nlarge > 0) hipLaunchKernelGGL((LARGE_K<false, false>), g1, blk, 0, ST, A);               \
        }                                                                                                     \
    } while (0)

void launch_sweep_count(const SweepArgs& a, hipStream_t st)
{
    if (a.g.nslots <= 0) return;
    DEM_SWEEP_LAUNCH(k_sweep_count, k_sweep_count_large, a, st);
}

void launch_sweep_fill(const SweepArgs& a, hipStream_t st)
{
    if (a.g.nslots <= 0) return;
    DEM_SWEEP_LAUNCH(k_sweep_fill_staged, k_sweep_fill_large, a, st);
    if (a.nent > 0) hipLaunchKernelGGL(k_row_rank, dim3(nblocks(a.nent)), dim3(kBlock), 0, st, a);
    if (a.nlarge > 0)
        hipLaunchKernelGGL(k_row_rank_large, dim3((a.nlarge + kBlock / 64 - 1) / (kBlock / 64)), dim3(kBlock), 0, st,
                           a);
}

void launch_pair_build(const PairBuildArgs& a, hipStream_t st)
{
    if (a.nent <= 0) return;
    hipLaunchKernelGGL(k_pair_build, dim3(nblocks(a.nent)), dim3(kBlock), 0, st, a);
}

void launch_carry_find(const PairBuildArgs& a, hipStream_t st, int old_nbodies)
{
    hipLaunchKernelGGL(k_carry_find, dim3(nblocks((long)a.npairs + 1)), dim3(kBlock), 0, st, a, old_nbodies);
}

void launch_partition(const PairBuildArgs& a, hipStream_t st)
{
    if (a.npairs > 0) hipLaunchKernelGGL(k_partition, dim3(nblocks(a.npairs)), dim3(kBlock), 0, st, a);
    if (a.nent > 0) hipLaunchKernelGGL(k_remap_rows, dim3(nblocks(a.nent)), dim3(kBlock), 0, st, a);
}

}  // namespace dem
