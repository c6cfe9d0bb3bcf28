// integrate.hip -- ForceContainer sum + NewtonIntegrator (section 2.1.5).
//
// One thread per body: the body adds the forces of its candidate pairs one by
// one, in ascending partner id (its row order; the wave helps with the
// gathers of a long row), so the sum is deterministic and needs no atomics;
// then gravity (damped like any force, dampGravity),
// Cundall damping eq. 2.9 per component with the on-step velocity estimate
// v + a dt/2, the leapfrog update, the spherical rotation and, in a periodic
// cell, the homoDeform velocity terms (class Cell).  Energies use the
// mid-step velocities v-, w-.  Each body also accumulates its non-affine
// displacement since the last broad-phase run and raises the step's stall
// flag once it exceeds the Verlet budget (eq. 2.3-2.4).  Energies go to the
// block's own slot; a periodic cell is updated, F+ = (I + L dt) F, by a
// one-block kernel after the step.
#include "dem_internal.hpp"

namespace dem {

namespace {

constexpr int kMaxBlock = 1024;

__device__ inline int logical_block(int nb)
{
    const int b = blockIdx.x;
    const int xcd = b & 7, idx = b >> 3;
    const int q = nb >> 3, r = nb & 7;
    return xcd * q + (xcd < r ? xcd : r) + idx;
}

__device__ inline double sgn(double x) { return x > 0.0 ? 1.0 : (x < 0.0 ? -1.0 : 0.0); }

// One touching pair as a row entry sees it: the force on #2 and n x F, from
// the pair's force record (FREC: F on #2, n x F) or from its history record
// (FP64 linear law: F = fn n + Fs).  Without contraction, so that every
// walk over a row (one thread, or the wave together) gives the same bits.
template <int PREC, bool FREC>
__device__ inline void pair_force(const StepArgs& a, uint32_t k, double* f)
{
#pragma clang fp contract(off)
    if (!FREC) {
        // the history record, one 64-byte segment read as two halves
        const gptr<const double4> h = glb<const double4>(reinterpret_cast<const double4*>(a.pr.h)) + 2 * (size_t)k;
        const double4 h0 = h[0], h1 = h[1];
        const double fx = h1.w * h1.x + h0.x, fy = h1.w * h1.y + h0.y, fz = h1.w * h1.z + h0.z;
        f[0] = fx;
        f[1] = fy;
        f[2] = fz;
        f[3] = h1.y * fz - h1.z * fy;
        f[4] = h1.z * fx - h1.x * fz;
        f[5] = h1.x * fy - h1.y * fx;
    } else if (PREC == DEM_FP32_MIXED) {
        // a record is read as three pairs (it starts on an 8-byte boundary)
        const gptr<const float2> q = glb<const float2>(reinterpret_cast<const float2*>(a.pr.frecf)) + 3 * (size_t)k;
        for (int c = 0; c < 3; ++c) {
            const float2 v = q[c];
            f[2 * c] = v.x;
            f[2 * c + 1] = v.y;
        }
    } else {
        const gptr<const double2> q = glb<const double2>(reinterpret_cast<const double2*>(a.pr.frec)) + 3 * (size_t)k;
        for (int c = 0; c < 3; ++c) {
            const double2 v = q[c];
            f[2 * c] = v.x;
            f[2 * c + 1] = v.y;
        }
    }
}

// Adds one touching entry to the body's sums: the force negated where the
// body is #1; both bodies of a pair feel -r_k (n x F) (lever arms r1 n and
// -r2 n).
__device__ inline void add_entry(uint32_t u, const double* f, double r, double* F, double* T)
{
#pragma clang fp contract(off)
    if (u & kNegSign) {
        F[0] += -f[0];
        F[1] += -f[1];
        F[2] += -f[2];
    } else {
        F[0] += f[0];
        F[1] += f[1];
        F[2] += f[2];
    }
    T[0] += -r * f[3];
    T[1] += -r * f[4];
    T[2] += -r * f[5];
}

// Entries [beg, end) of a row, added in row order (ascending partner id):
// taken four at a time so that their loads are in flight together (no
// branch between them: a position past the end reads the last entry again
// and is then ignored).  An entry carries its pair's touched bit.
template <int PREC, bool FREC>
__device__ inline void row_walk(const StepArgs& a, int beg, int end, double r, double* F, double* T)
{
    const gptr<const uint32_t> ent = glb<const uint32_t>(a.rows.ent);
    constexpr int kB = 4;
    for (int e0 = beg; e0 < end; e0 += kB) {
        uint32_t u[kB];
        bool use[kB];
        for (int j = 0; j < kB; ++j) u[j] = ent[min(e0 + j, end - 1)];
        for (int j = 0; j < kB; ++j) {
            const uint32_t k = u[j] & kPairMask;
            use[j] = (e0 + j < end) && k < (uint32_t)a.npairs && (u[j] & kRealBit) != 0u;
        }
        // the four gathers go out together, with no branch between them: an
        // entry that does not count reads pair 0's record (always cached)
        // and is then ignored
        double f[kB][kForceWords];
        for (int j = 0; j < kB; ++j) pair_force<PREC, FREC>(a, use[j] ? (u[j] & kPairMask) : 0u, f[j]);
        for (int j = 0; j < kB; ++j)
            if (use[j]) add_entry(u[j], f[j], r, F, T);
    }
}

// Resultant contact force and torque on a slot whose row is [beg, end), in
// row order: the forces of its touching pairs, negated where the body is #1.
template <int PREC, bool FREC>
__device__ inline void body_sum(const StepArgs& a, int beg, int end, double r, double* F, double* T)
{
    F[0] = F[1] = F[2] = 0.0;
    T[0] = T[1] = T[2] = 0.0;
    row_walk<PREC, FREC>(a, beg, end, r, F, T);
}

// The same sum in the integrate kernel, called by every lane of the wave.
// A lane walks at most kSoloEntries entries of its row by itself; longer
// rows (a large sphere among small ones has ~10x the entries of its
// neighbours, and its lane would hold the whole wave) are finished by the
// wave together, 64 entries at a time: each lane reads one entry and its
// pair's record into the wave's slice of LDS, then the row's own lane adds
// them in row order, with the same arithmetic as the walk.
constexpr int kSoloEntries = 12;
constexpr int kCoopWords = 64 * (kForceWords + 1);  // doubles per wave: 64 entries x 6, then 64 entry words
template <int PREC, bool FREC>
__device__ inline void body_sum_wave(const StepArgs& a, int beg, int end, double r, double* F, double* T,
                                     double* lds)
{
    F[0] = F[1] = F[2] = 0.0;
    T[0] = T[1] = T[2] = 0.0;
    const int solo = min(end, beg + kSoloEntries);
    row_walk<PREC, FREC>(a, beg, solo, r, F, T);
    const int lane = threadIdx.x & 63;
    uint32_t* lu = reinterpret_cast<uint32_t*>(lds + 64 * kForceWords);
    int next = solo;
    for (;;) {
        const unsigned long long need = __ballot(next < end);
        if (need == 0ull) break;
        const int src = __builtin_ctzll(need);
        const int c0 = __shfl(next, src, 64), c1 = __shfl(end, src, 64);
        const int e = c0 + lane;
        uint32_t u = 0u;
        if (e < c1) u = glb<const uint32_t>(a.rows.ent)[e];
        const uint32_t k = u & kPairMask;
        const bool use = e < c1 && k < (uint32_t)a.npairs && (u & kRealBit) != 0u;
        double f[kForceWords];
        if (use) {
            pair_force<PREC, FREC>(a, k, f);
            for (int q = 0; q < kForceWords; ++q) lds[q * 64 + lane] = f[q];
        }
        lu[lane] = use ? u : 0u;
        // the wave's own LDS writes are complete before its lanes read them
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        if (lane == src) {
            const int n = min(64, c1 - c0);
            for (int j = 0; j < n; ++j) {
                const uint32_t uj = lu[j];
                if (!(uj & kRealBit)) continue;
                double fj[kForceWords];
                for (int q = 0; q < kForceWords; ++q) fj[q] = lds[q * 64 + j];
                add_entry(uj, fj, r, F, T);
            }
            next = c0 + n;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
    }
}

__device__ inline void matvec(const double* M, double x, double y, double z, double* o)
{
    o[0] = (M[0] * x + M[1] * y) + M[2] * z;
    o[1] = (M[3] * x + M[4] * y) + M[5] * z;
    o[2] = (M[6] * x + M[7] * y) + M[8] * z;
}

struct IntPartial {
    double kin, rot, grav, damp, fsum, fcnt;
};

template <int PREC, bool BATCHED, bool PERIODIC, bool FREC>
__global__ void __launch_bounds__(kMaxBlock) k_integrate(const StepArgs* __restrict__ args, int parity)
{
    const StepArgs& a = *args;
    const int i = logical_block(gridDim.x) * blockDim.x + threadIdx.x;
    const bool live = i < a.nslots;
    const gptr<double4> bxr = glb(a.bod.xr), bvm = glb(a.bod.vm), bw = glb(a.bod.w), bq = glb(a.bod.q);
    // the previous step's stall flag is read first and tested only after the
    // body's loads are issued (they are in bounds, and nothing is stored
    // before the test), so that its latency overlaps theirs; the row bounds
    // before the body state: the row's loads wait for them
    const int32_t stalled = a.ctr->stall[parity ^ 1];
    int beg = 0, end = 0;
    double4 xr0 = make_double4(0.0, 0.0, 0.0, 0.0), vm0 = xr0, w0 = xr0;
    uint16_t mi = 0;
    uint8_t blocked = 0;
    if (live) {
        beg = glb<const int32_t>(a.rows.start)[i];
        end = glb<const int32_t>(a.rows.start)[i + 1];
        xr0 = bxr[i];
        vm0 = bvm[i];
        w0 = bw[i];
        mi = glb<const uint16_t>(a.bod.mat)[i];
        blocked = glb<const uint8_t>(a.bod.blocked)[i];
    }
    if (stalled) {
        // not run: keep every later step of this launch chain stopped too
        if (blockIdx.x == 0 && threadIdx.x == 0) a.ctr->stall[parity] = 1;
        return;
    }
    // this step ends an update period of the controlled cell: also sum the
    // dynamic spheres' |resultant contact force| (unbalanced force)
    const bool measure = a.ctr->measure != 0;
    IntPartial part = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    bool bad = false;
    bool over = false;
    // the contact force sum, by every lane of the wave (a lane past the last
    // body has an empty row)
    extern __shared__ double s_coop[];
    double F[3], T[3];
    body_sum_wave<PREC, FREC>(a, beg, end, xr0.w, F, T, s_coop + (threadIdx.x >> 6) * kCoopWords);
    if (live) {
        const int s = BATCHED ? (int)glb<const uint16_t>(a.bod.scene)[i] : 0;
        // an unbatched scene (periodic included) reads the descriptor's own
        // copy of its parameters: uniform, read-only here, so scalar loads
        const SceneParams& S = BATCHED ? a.scenes[s] : a.scene0;
        const double dt = S.dt;
        const double lam = S.damping;
        const double rho = glb<const Material>(a.mats)[mi].density;
        const double r = xr0.w, m = sphere_mass(r, rho);
        const double I = 2.0 * m * r * r / 5.0;
        // FP64 division costs about ten FP64 instructions: the step divides
        // by m and by I once and multiplies after that
        const double inv_m = 1.0 / m, inv_I = 1.0 / I;
        if (measure && blocked != 63u) {
            part.fsum = sqrt(F[0] * F[0] + F[1] * F[1] + F[2] * F[2]);
            part.fcnt = 1.0;
        }

        const double x0[3] = {xr0.x, xr0.y, xr0.z};
        const double v0[3] = {vm0.x, vm0.y, vm0.z};
        double w[3] = {w0.x, w0.y, w0.z};
        double f[3], t[3];
        for (int k = 0; k < 3; ++k) {
            f[k] = F[k] + m * S.gravity[k];
            t[k] = T[k];
        }
        part.kin = 0.5 * m * ((v0[0] * v0[0] + v0[1] * v0[1]) + v0[2] * v0[2]);
        part.rot = 0.5 * I * ((w[0] * w[0] + w[1] * w[1]) + w[2] * w[2]);

        double homo[3] = {0.0, 0.0, 0.0};
        if (PERIODIC && S.homo_deform > 0) {
            double dL[9], a1[3], a2[3];
            for (int k = 0; k < 9; ++k) dL[k] = S.L[k] - S.Lprev[k];
            matvec(dL, x0[0], x0[1], x0[2], a1);
            matvec(S.L, v0[0], v0[1], v0[2], a2);
            for (int k = 0; k < 3; ++k) homo[k] = a1[k] + (S.homo_deform == 2 ? a2[k] * dt : 0.0);
        }
        double v[3];
        for (int k = 0; k < 3; ++k) {
            if (blocked & (1u << k)) {
                v[k] = v0[k];
                continue;
            }
            part.grav += -m * S.gravity[k] * v0[k] * dt;
            if (lam > 0.0) {
                const double acc = f[k] * inv_m;
                const double df = -lam * sgn(f[k] * (v0[k] + acc * dt / 2.0)) * f[k];
                part.damp += -df * v0[k] * dt;
                f[k] += df;
            }
            v[k] = v0[k] + f[k] * inv_m * dt + homo[k];
        }
        const double x1[3] = {x0[0] + v[0] * dt, x0[1] + v[1] * dt, x0[2] + v[2] * dt};

        for (int k = 0; k < 3; ++k) {
            if (blocked & (8u << k)) continue;
            if (lam > 0.0 && S.damp_rot) {
                // the torque's share of the damping work uses the mid-step spin
                const double acc = t[k] * inv_I;
                const double dtq = -lam * sgn(t[k] * (w[k] + acc * dt / 2.0)) * t[k];
                part.damp += -dtq * w[k] * dt;
                t[k] += dtq;
            }
            w[k] = w[k] + t[k] * inv_I * dt;
        }
        const double ww = (w[0] * w[0] + w[1] * w[1]) + w[2] * w[2];
        if (ww > 0.0) {
            // the orientation only changes (and is only read) for a spinning body
            const double wn = sqrt(ww);
            const double4 q0 = bq[i];
            double q[4] = {q0.x, q0.y, q0.z, q0.w};
            const double half = 0.5 * wn * dt;
            const double sh = sin(half) / wn;
            const double d0 = cos(half), d1 = w[0] * sh, d2 = w[1] * sh, d3 = w[2] * sh;
            const double n0 = d0 * q[0] - d1 * q[1] - d2 * q[2] - d3 * q[3];
            const double n1 = d0 * q[1] + d1 * q[0] + d2 * q[3] - d3 * q[2];
            const double n2 = d0 * q[2] - d1 * q[3] + d2 * q[0] + d3 * q[1];
            const double n3 = d0 * q[3] + d1 * q[2] - d2 * q[1] + d3 * q[0];
            const double inv_qn = 1.0 / sqrt(n0 * n0 + n1 * n1 + n2 * n2 + n3 * n3);
            q[0] = n0 * inv_qn;
            q[1] = n1 * inv_qn;
            q[2] = n2 * inv_qn;
            q[3] = n3 * inv_qn;
            bq[i] = make_double4(q[0], q[1], q[2], q[3]);
        }
        bxr[i] = make_double4(x1[0], x1[1], x1[2], r);
        // the Verlet account (fourth word of vm): non-affine displacement of
        // this step (eq. 2.3); the cell's mean field uses its own share
        double u[3] = {v[0], v[1], v[2]};
        if (PERIODIC) {
            double Lx[3];
            matvec(S.L, x0[0], x0[1], x0[2], Lx);
            for (int k = 0; k < 3; ++k) u[k] -= Lx[k];
        }
        const double d = vm0.w + sqrt((u[0] * u[0] + u[1] * u[1]) + u[2] * u[2]) * dt + a.ctr->verlet_cell_step;
        bvm[i] = make_double4(v[0], v[1], v[2], d);
        // an unchanged spin (no torque, or blocked) is not stored again
        if (w[0] != w0.x || w[1] != w0.y || w[2] != w0.z) bw[i] = make_double4(w[0], w[1], w[2], 0.0);

        over = d > a.ctr->verlet_limit;
        bad = !(isfinite(x1[0]) && isfinite(x1[1]) && isfinite(x1[2]) && isfinite(v[0]) && isfinite(v[1]) &&
                isfinite(v[2]));
    }
    // eq. 2.4: some body may now have left its enlarged bound: the next step
    // needs a broad-phase run (plain stores of the same value)
    if (__any(over) && (threadIdx.x & 63) == 0) a.ctr->stall[parity] = 1;
    if (__any(bad) && (threadIdx.x & 63) == 0) a.ctr->nonfinite = 1;
    if (blockIdx.x == 0 && threadIdx.x == 0) a.ctr->steps_done += 1;
    const bool energy = a.track_energy != 0;
    if (!energy && !measure) return;

    // ---- energies and the controlled cell's force sums into this block's
    // slot (fixed-order wave/block sums)
    __shared__ IntPartial s_p[kMaxBlock / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    for (int off = 32; off > 0; off >>= 1) {
        if (energy) {
            part.kin += __shfl_down(part.kin, off, 64);
            part.rot += __shfl_down(part.rot, off, 64);
            part.grav += __shfl_down(part.grav, off, 64);
            part.damp += __shfl_down(part.damp, off, 64);
        }
        if (measure) {
            part.fsum += __shfl_down(part.fsum, off, 64);
            part.fcnt += __shfl_down(part.fcnt, off, 64);
        }
    }
    if (lane == 0) s_p[wave] = part;
    __syncthreads();
    if (threadIdx.x == 0) {
        IntPartial p = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        for (int w = 0; w < nwaves; ++w) {
            p.kin += s_p[w].kin;
            p.rot += s_p[w].rot;
            p.grav += s_p[w].grav;
            p.damp += s_p[w].damp;
            p.fsum += s_p[w].fsum;
            p.fcnt += s_p[w].fcnt;
        }
        IntAcc& acc = a.acc_integrate[blockIdx.x];
        if (energy) {
            acc.kin = p.kin;
            acc.rot = p.rot;
            acc.grav += p.grav;
            acc.damp += p.damp;
        }
        if (measure) {
            acc.fsum = p.fsum;
            acc.fcnt = p.fcnt;
        }
    }
}

// The controlled cell's first reduction level (update steps only): block g
// of kCtrlReduceGrid sums, in a fixed order, a fixed contiguous share of the
// contact kernel's per-block terms (term-major in acc_ctrl) and of the
// integrate kernel's slots, into kCtrlWords values at acc_ctrl2[g].
constexpr int kCtrlWords = kNetworkWords + 2;
constexpr int kCtrlReduceBlock = 256;

__global__ void __launch_bounds__(kCtrlReduceBlock) k_ctrl_reduce(const StepArgs* __restrict__ args, int parity)
{
    const StepArgs& a = *args;
    if (a.ctr->stall[parity ^ 1] || !a.ctr->measure) return;
    const int g = blockIdx.x, G = gridDim.x;
    const int nb = a.nblocks_contact, ni = a.nblocks_integrate;
    const int b0 = (int)(((int64_t)g * nb) / G), b1 = (int)(((int64_t)(g + 1) * nb) / G);
    const int i0 = (int)(((int64_t)g * ni) / G), i1 = (int)(((int64_t)(g + 1) * ni) / G);
    double t[kCtrlWords];
    for (int q = 0; q < kCtrlWords; ++q) t[q] = 0.0;
    for (int b = b0 + (int)threadIdx.x; b < b1; b += blockDim.x)
        for (int q = 0; q < kNetworkWords; ++q) t[q] += a.acc_ctrl[(size_t)q * nb + b];
    for (int i = i0 + (int)threadIdx.x; i < i1; i += blockDim.x) {
        t[kNetworkWords] += a.acc_integrate[i].fsum;
        t[kNetworkWords + 1] += a.acc_integrate[i].fcnt;
    }
    __shared__ double sh[kCtrlReduceBlock / 64][kCtrlWords];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int q = 0; q < kCtrlWords; ++q)
        for (int off = 32; off > 0; off >>= 1) t[q] += __shfl_down(t[q], off, 64);
    if (lane == 0)
        for (int q = 0; q < kCtrlWords; ++q) sh[wave][q] = t[q];
    __syncthreads();
    if (threadIdx.x < kCtrlWords) {
        double v = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) v += sh[w][threadIdx.x];
        a.acc_ctrl2[(size_t)kCtrlWords * g + threadIdx.x] = v;
    }
}

// Periodic cell (section 2.1.6), once per step after the bodies: H+ =
// (I + L dt) H and the same for trsf; H - H_prev is kept for the image
// velocity of the next step's contacts; L becomes L_prev.  Then, on the
// steps that end an update period of the controlled cell, the controller
// (PeriTriaxController driven by the packing stiffness) sets the velocity
// gradient of the next steps from the partial sums of the contact kernel's
// measuring instantiation and of the integrate kernel's slots (first reduced
// by k_ctrl_reduce): per stress axis (1 - grow_damping)(goal - sigma_ii)/(M_i T),
// M_i = (1/V) sum k_n (d_i n_i)^2 and T = glob_update dt (the full rate
// towards the goal's sign while M_i = 0), per strain axis
// (goal - log trsf_ii)/T, capped at max_rate; zero once the goal is reached
// (every stress axis within max(abs_tol, rel_tol |goal|), every strain axis
// within 1e-6, unbalanced force at most max_unbalanced), and with
// stop_when_done the launch chain halts.  One block; the partial sums are
// combined in a fixed order (a fixed range per thread, then a fixed tree).
constexpr int kCellBlock = 256;

__global__ void __launch_bounds__(kCellBlock) k_cell_update(StepArgs* args, int parity)
{
    const StepArgs& a = *args;
    if (a.ctr->stall[parity ^ 1]) return;
    SceneParams* S = &a.scenes[0];
    if (threadIdx.x == 0) {
        const double dt = S->dt;
        double M[9], Hn[9], Tn[9];
        for (int k = 0; k < 9; ++k) M[k] = ((k % 4 == 0) ? 1.0 : 0.0) + S->L[k] * dt;
        for (int r = 0; r < 3; ++r)
            for (int q = 0; q < 3; ++q) {
                Hn[3 * r + q] = (M[3 * r + 0] * S->H[q] + M[3 * r + 1] * S->H[3 + q]) + M[3 * r + 2] * S->H[6 + q];
                Tn[3 * r + q] =
                    (M[3 * r + 0] * S->trsf[q] + M[3 * r + 1] * S->trsf[3 + q]) + M[3 * r + 2] * S->trsf[6 + q];
            }
        for (int k = 0; k < 9; ++k) {
            S->dH[k] = Hn[k] - S->H[k];
            S->H[k] = Hn[k];
            S->trsf[k] = Tn[k];
            S->Lprev[k] = S->L[k];
        }
        const double* A = S->H;
        const double a0 = A[0], a1 = A[1], a2 = A[2], a3 = A[3], a4 = A[4], a5 = A[5], a6 = A[6], a7 = A[7],
                     a8 = A[8];
        const double C0 = a4 * a8 - a5 * a7, C1 = -(a3 * a8 - a5 * a6), C2 = a3 * a7 - a4 * a6;
        const double det = a0 * C0 + a1 * C1 + a2 * C2;
        S->Hinv[0] = C0 / det;
        S->Hinv[1] = -(a1 * a8 - a2 * a7) / det;
        S->Hinv[2] = (a1 * a5 - a2 * a4) / det;
        S->Hinv[3] = C1 / det;
        S->Hinv[4] = (a0 * a8 - a2 * a6) / det;
        S->Hinv[5] = -(a0 * a5 - a2 * a3) / det;
        S->Hinv[6] = C2 / det;
        S->Hinv[7] = -(a0 * a7 - a1 * a6) / det;
        S->Hinv[8] = (a0 * a4 - a1 * a3) / det;
    }
    const CtrlConfig& c = *a.ctrl;
    if (c.active && a.ctr->measure) {
        // fixed-order sum of the partials: thread t takes the blocks t,
        // t + blockDim, ... in order; then a fixed pairwise tree over threads
        constexpr int W = kCtrlWords;
        double t[W];
        for (int q = 0; q < W; ++q) t[q] = 0.0;
        for (int g = threadIdx.x; g < kCtrlReduceGrid; g += blockDim.x)
            for (int q = 0; q < W; ++q) t[q] += a.acc_ctrl2[(size_t)W * g + q];
        __shared__ double sh[kCellBlock][W];
        for (int q = 0; q < W; ++q) sh[threadIdx.x][q] = t[q];
        __syncthreads();
        for (int half = kCellBlock / 2; half > 0; half >>= 1) {
            if ((int)threadIdx.x < half)
                for (int q = 0; q < W; ++q) sh[threadIdx.x][q] += sh[threadIdx.x + half][q];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            const double* sum = sh[0];
            CtrlState& st = *a.ctrl_state;
            const double* H = S->H;
            const double V = fabs(H[0] * (H[4] * H[8] - H[5] * H[7]) - H[1] * (H[3] * H[8] - H[5] * H[6]) +
                                  H[2] * (H[3] * H[7] - H[4] * H[6]));
            const double T = (double)c.glob_update * S->dt;
            double rates[3];
            bool reached = true;
            const double ncont = sum[13], ndyn = sum[kNetworkWords + 1];
            st.unbalanced = (ncont > 0.0 && ndyn > 0.0) ? (sum[kNetworkWords] / ndyn) / (sum[12] / ncont) : NAN;
            for (int i = 0; i < 3; ++i) {
                st.stress[i] = sum[4 * i] / V;
                st.strain[i] = log(S->trsf[4 * i]);
                st.stiff[i] = sum[9 + i] / V;
            }
            if (c.iso) {
                // the isotropic compressor: mean stress and mean modulus, one
                // rate; a reached stress (balanced packing) hands over to the
                // next of the series in the same update
                const double sm = (st.stress[0] + st.stress[1] + st.stress[2]) / 3.0;
                const double Mm = (st.stiff[0] + st.stiff[1] + st.stiff[2]) / 3.0;
                double goal = c.series[st.series_index];
                auto at_goal = [&](double g) {
                    return fabs(g - sm) <= fmax(c.abs_tol, c.rel_tol * fabs(g)) && st.unbalanced <= c.max_unbalanced;
                };
                reached = at_goal(goal);
                if (reached && st.series_index + 1 < c.n_series) {
                    st.series_index += 1;
                    goal = c.series[st.series_index];
                    reached = false;
                }
                const double err = goal - sm;
                double rate;
                if (Mm > 0.0)
                    rate = (1.0 - c.grow_damping) * err / (Mm * T);
                else
                    rate = err != 0.0 ? copysign(c.max_rate[0], err) : 0.0;
                rate = fmax(-c.max_rate[0], fmin(c.max_rate[0], rate));
                rates[0] = rates[1] = rates[2] = rate;
            }
            for (int i = 0; i < 3 && !c.iso; ++i) {
                double rate;
                if (c.stress_mask & (1 << i)) {
                    const double err = c.goal[i] - st.stress[i];
                    if (st.stiff[i] > 0.0)
                        rate = (1.0 - c.grow_damping) * err / (st.stiff[i] * T);
                    else
                        rate = err != 0.0 ? copysign(c.max_rate[i], err) : 0.0;
                    if (fabs(err) > fmax(c.abs_tol, c.rel_tol * fabs(c.goal[i]))) reached = false;
                } else {
                    const double err = c.goal[i] - st.strain[i];
                    rate = err / T;
                    if (fabs(err) > 1e-6) reached = false;
                }
                rates[i] = fmax(-c.max_rate[i], fmin(c.max_rate[i], rate));
            }
            if (!c.iso && !(st.unbalanced <= c.max_unbalanced)) reached = false;
            st.done = reached ? 1 : 0;
            if (reached) rates[0] = rates[1] = rates[2] = 0.0;
            double lf = 0.0;
            for (int k = 0; k < 9; ++k) S->L[k] = 0.0;
            for (int i = 0; i < 3; ++i) {
                st.rate[i] = rates[i];
                S->L[4 * i] = rates[i];
                lf += rates[i] * rates[i];
            }
            st.updates += 1;
            // the mean field's share of the Verlet budget follows the new gradient
            S->verlet_cell_rate = 0.5 * sqrt(lf) * (2.0 * S->rmax + 4.0 * S->verlet);
            a.ctr->verlet_cell_step = S->verlet_cell_rate * S->dt;
            if (reached && c.stop_when_done) {
                a.ctr->halt = 1;
                a.ctr->stall[parity] = 1;  // the remaining steps of the chain do not run
            }
        }
    }
    // the step kernels of an unbatched scene read the descriptor's copy
    if (threadIdx.x == 0) args->scene0 = *S;
}

// Resultant force/torque per slot (for reporting), same sum as the step.
template <int PREC, bool FREC>
__global__ void k_body_forces(StepArgs a, double* __restrict__ f3, double* __restrict__ t3)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.nslots) return;
    double F[3], T[3];
    body_sum<PREC, FREC>(a, a.rows.start[i], a.rows.start[i + 1], a.bod.xr[i].w, F, T);
    for (int k = 0; k < 3; ++k) {
        f3[3 * i + k] = F[k];
        t3[3 * i + k] = T[k];
    }
}

// Per-body measures of one scene for the unbalanced force and the stiffness
// timestepper (reporting, not in the step), kBodyWords doubles per block:
// sum and largest |resultant contact force| over the dynamic spheres (not
// all six DOFs blocked), their number, and the smallest critical timestep
// sqrt(2) sqrt(m / K_ii) over their unblocked DOFs (eq. 2.12), with the
// translational stiffness K_ii = sum of (k_n - k_s) n_i^2 + k_s over the
// body's contacts (eq. 2.14) and the rotational one R_ii = sum of
// k_s r^2 (1 - n_i^2) against the inertia (+inf without contacts).
constexpr int kMeasureBlock = 256;

template <int PREC, bool BATCHED, bool FREC>
__global__ void __launch_bounds__(kMeasureBlock) k_body_measures(StepArgs a, int scene, double* __restrict__ part)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double fsum = 0.0, fmaxv = 0.0, cnt = 0.0, dtmin = INFINITY;
    if (i < a.nslots && (!BATCHED || (int)a.bod.scene[i] == scene) && a.bod.blocked[i] != 63u) {
        const unsigned blocked = a.bod.blocked[i];
        const double4 xr = a.bod.xr[i];
        const double r = xr.w, m = sphere_mass(r, a.mats[a.bod.mat[i]].density);
        const double I = 2.0 * m * r * r / 5.0;
        const int beg = a.rows.start[i], end = a.rows.start[i + 1];
        double F[3], T[3];
        body_sum<PREC, FREC>(a, beg, end, r, F, T);
        const double fa = sqrt(F[0] * F[0] + F[1] * F[1] + F[2] * F[2]);
        fsum = fa;
        fmaxv = fa;
        cnt = 1.0;
        double K[3] = {0.0, 0.0, 0.0}, Rr[3] = {0.0, 0.0, 0.0};
        for (int e = beg; e < end; ++e) {
            const uint32_t k = a.rows.ent[e] & kPairMask;
            if (!a.pr.real[k]) continue;
            const HistRec h = hist_load<PREC>(a.pr.h, k);
            const double n[3] = {h.nx, h.ny, h.nz};
            const int sa = a.pr.a[k], sb = a.pr.b[k];
            const bool wall = sa < 0;
            const double r2 = a.bod.xr[sb].w;
            const double r1 = wall ? (a.walls[-1 - sa].kind == kFacet ? 2.0 * r2 : r2) : a.bod.xr[sa].w;
            const int m1 = wall ? a.walls[-1 - sa].mat : (int)a.bod.mat[sa];
            const Material M1 = a.mats[m1], M2 = a.mats[a.bod.mat[sb]];
            const double k1 = M1.young * (2.0 * r1), k2 = M2.young * (2.0 * r2);
            const double kn = k1 * k2 / (k1 + k2);
            const double q1 = M1.young_poisson * (2.0 * r1), q2 = M2.young_poisson * (2.0 * r2);
            const double ks = q1 * q2 / (q1 + q2);
            for (int c = 0; c < 3; ++c) {
                K[c] += (kn - ks) * n[c] * n[c] + ks;
                Rr[c] += ks * r * r * (1.0 - n[c] * n[c]);
            }
        }
        for (int c = 0; c < 3; ++c) {
            if (!(blocked & (1u << c)) && K[c] > 0.0) dtmin = fmin(dtmin, sqrt(2.0) * sqrt(m / K[c]));
            if (!(blocked & (8u << c)) && Rr[c] > 0.0) dtmin = fmin(dtmin, sqrt(2.0) * sqrt(I / Rr[c]));
        }
    }
    __shared__ double sh[kMeasureBlock / 64][kBodyWords];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int off = 32; off > 0; off >>= 1) {
        fsum += __shfl_down(fsum, off, 64);
        fmaxv = fmax(fmaxv, __shfl_down(fmaxv, off, 64));
        cnt += __shfl_down(cnt, off, 64);
        dtmin = fmin(dtmin, __shfl_down(dtmin, off, 64));
    }
    if (lane == 0) {
        sh[wave][0] = fsum;
        sh[wave][1] = fmaxv;
        sh[wave][2] = cnt;
        sh[wave][3] = dtmin;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t[kBodyWords] = {0.0, 0.0, 0.0, INFINITY};
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
            t[0] += sh[w][0];
            t[1] = fmax(t[1], sh[w][1]);
            t[2] += sh[w][2];
            t[3] = fmin(t[3], sh[w][3]);
        }
        for (int q = 0; q < kBodyWords; ++q) part[kBodyWords * (size_t)blockIdx.x + q] = t[q];
    }
}

template <int PREC, bool BATCHED, bool PERIODIC, bool FREC>
void launch_t(const StepArgs* args, int parity, int grid, int block, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1)
{
    const dim3 g(grid > 0 ? grid : 1), b(block);
    // each wave's LDS slice for the long rows' cooperative walk
    const size_t lds = sizeof(double) * kCoopWords * (size_t)((block + 63) / 64);
    if (ev0)
        hipExtLaunchKernelGGL((k_integrate<PREC, BATCHED, PERIODIC, FREC>), g, b, lds, st, ev0, ev1, 0, args, parity);
    else
        hipLaunchKernelGGL((k_integrate<PREC, BATCHED, PERIODIC, FREC>), g, b, lds, st, args, parity);
}

template <int PREC, bool FREC>
void launch_kind(const StepArgs* args, int parity, int grid, bool batched, bool periodic, int block, hipStream_t st,
                 hipEvent_t ev0, hipEvent_t ev1)
{
    if (batched) launch_t<PREC, true, false, FREC>(args, parity, grid, block, st, ev0, ev1);
    else if (periodic) launch_t<PREC, false, true, FREC>(args, parity, grid, block, st, ev0, ev1);
    else launch_t<PREC, false, false, FREC>(args, parity, grid, block, st, ev0, ev1);
}

}  // namespace

void launch_integrate(const StepArgs* args, int parity, int grid, int precision, bool batched, bool periodic,
                      bool frec, int block, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1)
{
    // FP32-mixed always has its force records
    if (precision == DEM_FP32_MIXED)
        launch_kind<DEM_FP32_MIXED, true>(args, parity, grid, batched, periodic, block, st, ev0, ev1);
    else if (frec)
        launch_kind<DEM_FP64, true>(args, parity, grid, batched, periodic, block, st, ev0, ev1);
    else
        launch_kind<DEM_FP64, false>(args, parity, grid, batched, periodic, block, st, ev0, ev1);
}

// Largest Verlet account (non-affine displacement since the last broad-phase
// run, the fourth word of vm) over the bodies: wave maxima, then an integer
// maximum on the bits (non-negative doubles order like their bits).
__global__ void __launch_bounds__(256) k_max_account(Bodies b, int n, unsigned long long* __restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double v = i < n ? b.vm[i].w : 0.0;
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(out, (unsigned long long)__double_as_longlong(v));
}

void launch_max_account(const Bodies& b, int n, unsigned long long* out, hipStream_t st)
{
    if (n > 0) hipLaunchKernelGGL(k_max_account, dim3((n + 255) / 256), dim3(256), 0, st, b, n, out);
}

void launch_ctrl_reduce(const StepArgs* args, int parity, hipStream_t st)
{
    hipLaunchKernelGGL(k_ctrl_reduce, dim3(kCtrlReduceGrid), dim3(kCtrlReduceBlock), 0, st, args, parity);
}

void launch_cell_update(const StepArgs* args, int parity, hipStream_t st)
{
    hipLaunchKernelGGL(k_cell_update, dim3(1), dim3(kCellBlock), 0, st, const_cast<StepArgs*>(args), parity);
}


int body_blocks(int nslots) { return nslots > 0 ? (nslots + kMeasureBlock - 1) / kMeasureBlock : 0; }

void launch_body_measures(const StepArgs& a, int precision, bool batched, int scene, double* part, hipStream_t st)
{
    const int grid = body_blocks(a.nslots);
    if (grid == 0) return;
    const dim3 g(grid), b(kMeasureBlock);
    if (precision == DEM_FP32_MIXED) {
        if (batched) hipLaunchKernelGGL((k_body_measures<DEM_FP32_MIXED, true, true>), g, b, 0, st, a, scene, part);
        else hipLaunchKernelGGL((k_body_measures<DEM_FP32_MIXED, false, true>), g, b, 0, st, a, scene, part);
    } else if (a.use_frec) {
        if (batched) hipLaunchKernelGGL((k_body_measures<DEM_FP64, true, true>), g, b, 0, st, a, scene, part);
        else hipLaunchKernelGGL((k_body_measures<DEM_FP64, false, true>), g, b, 0, st, a, scene, part);
    } else {
        if (batched) hipLaunchKernelGGL((k_body_measures<DEM_FP64, true, false>), g, b, 0, st, a, scene, part);
        else hipLaunchKernelGGL((k_body_measures<DEM_FP64, false, false>), g, b, 0, st, a, scene, part);
    }
}

void launch_body_forces(const StepArgs& a, int precision, double* f3, double* t3, hipStream_t st)
{
    if (a.nslots <= 0) return;
    const int grid = (a.nslots + 255) / 256;
    if (precision == DEM_FP32_MIXED)
        hipLaunchKernelGGL((k_body_forces<DEM_FP32_MIXED, true>), dim3(grid), dim3(256), 0, st, a, f3, t3);
    else if (a.use_frec)
        hipLaunchKernelGGL((k_body_forces<DEM_FP64, true>), dim3(grid), dim3(256), 0, st, a, f3, t3);
    else
        hipLaunchKernelGGL((k_body_forces<DEM_FP64, false>), dim3(grid), dim3(256), 0, st, a, f3, t3);
}

}  // namespace dem
