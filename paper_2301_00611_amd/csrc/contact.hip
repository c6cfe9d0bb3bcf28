// contact.hip -- the InteractionLoop for one fixed set of functors: one
// thread per candidate pair runs the exact contact test, the ScGeom update
// (class ScGeom; section 2.1.3), Ip2_FrictMat_FrictMat_FrictPhys (section
// 2.1.2) and Law2_ScGeom_FrictPhys_CundallStrack (section 2.1.4), and writes
// the pair's history record (shear force, normal, overlap, normal force),
// plus a force record (force on #2, n x F) in FP32-mixed mode and under the
// visco-elastic law.  No sum happens here: each body adds its pairs' forces
// later, in a fixed order (integrate.hip).
//
// FP64 mode computes everything in double.  FP32-mixed mode keeps the
// contact test, the branch length and the overlap in double (they are
// differences of absolute positions), then evaluates the normal, the
// relative velocity, the stiffnesses and the forces in float; the shear
// force history stays double (the float increment is added to it).
#include "dem_internal.hpp"

namespace dem {

namespace {

constexpr int kMaxBlock = 1024;

template <typename T>
struct V3 {
    T x, y, z;
};
template <typename T>
__device__ inline V3<T> v3(T x, T y, T z) { return {x, y, z}; }
template <typename T>
__device__ inline V3<T> operator+(V3<T> a, V3<T> b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <typename T>
__device__ inline V3<T> operator-(V3<T> a, V3<T> b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <typename T>
__device__ inline V3<T> operator*(T s, V3<T> a) { return {s * a.x, s * a.y, s * a.z}; }
template <typename T>
__device__ inline T dot(V3<T> a, V3<T> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <typename T>
__device__ inline V3<T> cross(V3<T> a, V3<T> b)
{
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <typename T, typename U>
__device__ inline V3<T> cvt(V3<U> a) { return {(T)a.x, (T)a.y, (T)a.z}; }

// The exact contact test of two spheres: |d|^2 < (r1 + r2)^2 with
// d = (x2 + H c) - x1, evaluated left to right with no fused multiply-add,
// so that the pair set is identical bit for bit to a plain FP64 evaluation.
struct SpherePairTest {
    double dx, dy, dz, dd;
    bool real;
};
template <bool PERIODIC>
__device__ inline SpherePairTest sphere_pair_test(double x1, double y1, double z1, double x2,
                                                                      double y2, double z2, double r1, double r2,
                                                                      const double* H, int cx, int cy, int cz)
{
#pragma clang fp contract(off)
    SpherePairTest t;
    if (PERIODIC) {
        const double sx = (H[0] * (double)cx + H[1] * (double)cy) + H[2] * (double)cz;
        const double sy = (H[3] * (double)cx + H[4] * (double)cy) + H[5] * (double)cz;
        const double sz = (H[6] * (double)cx + H[7] * (double)cy) + H[8] * (double)cz;
        t.dx = (x2 + sx) - x1;
        t.dy = (y2 + sy) - y1;
        t.dz = (z2 + sz) - z1;
    } else {
        t.dx = x2 - x1;
        t.dy = y2 - y1;
        t.dz = z2 - z1;
    }
    t.dd = (t.dx * t.dx + t.dy * t.dy) + t.dz * t.dz;
    const double s = r1 + r2;
    t.real = t.dd < s * s;
    return t;
}

__device__ inline void unpack_cell(int32_t p, int* c)
{
    uint32_t u = (uint32_t)p;
    c[0] = (int)((u >> 20) & 1023u) - 512;
    c[1] = (int)((u >> 10) & 1023u) - 512;
    c[2] = (int)(u & 1023u) - 512;
}

// Blocks are dispatched round-robin over the 8 XCDs (block b runs on XCD
// b & 7).  Each XCD takes one eighth of the pairs, a contiguous segment
// [P_x, P_x+1) with P_x = x npairs / 8, so that neighbouring pairs share its
// L2 and every XCD gets the same share whatever the grid's headroom (the
// grid has at least ceil(ceil(npairs / 8) / blockDim) blocks per XCD).
// Returns the pair of this thread, or -1.
__device__ inline int xcd_pair(int npairs)
{
    const int xcd = blockIdx.x & 7, j = blockIdx.x >> 3;
    const int64_t p0 = ((int64_t)xcd * npairs) >> 3, p1 = ((int64_t)(xcd + 1) * npairs) >> 3;
    const int64_t k = p0 + (int64_t)j * blockDim.x + threadIdx.x;
    return k < p1 ? (int)k : -1;
}

// A pair that starts or stops touching rewrites its two row entries with
// the new touched bit (a boundary pair has only #2's), so that the force sum
// reads the state from the entry itself; the pair is #1's and adds -F there.
__device__ inline void set_row_bits(const StepArgs& a, int k, bool real)
{
    const gptr<uint32_t> ent = glb(a.rows.ent);
    const int32_t ea = glb<const int32_t>(a.pr.ea)[k], eb = glb<const int32_t>(a.pr.eb)[k];
    const uint32_t v = (uint32_t)k | (real ? kRealBit : 0u);
    if (ea >= 0) ent[ea] = v | kNegSign;
    if (eb >= 0) ent[eb] = v;
}

struct ContactPartial {
    double el, plast;
    unsigned long long ss, sw;
    double visc;
};

// MEASURE (periodic, unbatched; launched on the steps that end an update
// period of the controlled cell only): the kernel also sums, per block, the
// controller's contact terms: the Love-Weber stress (9, sphere pairs), the
// normal springs' modulus k_n (d_i n_i)^2 (3, sphere pairs; d = l n the
// centre distance vector) and |F| with a count (every touching pair), from
// the force and normal as stored.  A separate instantiation, so that the
// extra registers do not lower the occupancy of every other step.
// PRIMS (aperiodic scenes holding a box or a facet): the geometry of those
// boundaries is compiled in; without it the kernel keeps its registers for
// spheres and planes.
// VISCEL (a world with visco-elastic materials): pairs of ViscElMat take
// Law2_ScGeom_ViscElPhys_Basic, the others the linear law.
template <int PREC, bool BATCHED, bool PERIODIC, bool MEASURE = false, bool PRIMS = false, bool VISCEL = false>
__global__ void __launch_bounds__(kMaxBlock) k_contact(const StepArgs* __restrict__ args, int parity)
{
    using R = typename std::conditional<PREC == DEM_FP32_MIXED, float, double>::type;
    // the arguments live in device memory so that a captured graph stays
    // valid across broad-phase runs (pair count and buffers change there)
    const StepArgs& a = *args;
    // the previous step's stall flag is read first and tested only after this
    // thread's pair ids and its touched flag are requested (in bounds;
    // nothing is stored before the test), so that its latency overlaps theirs
    const int32_t stalled = a.ctr->stall[parity ^ 1];
    const int k = xcd_pair(a.npairs);
    int32_t sa = 0, sb = 0, pcell = 0;
    uint8_t was_real = 0;
    if (k >= 0) {
        sa = glb<const int32_t>(a.pr.a)[k];
        sb = glb<const int32_t>(a.pr.b)[k];
        if (PERIODIC) pcell = glb<const int32_t>(a.pr.cell)[k];
        was_real = glb<const uint8_t>(a.pr.real)[k];
    }
    // the previous step asked for a broad-phase run: this step does not run
    if (stalled) return;
    // this step's flag starts clear; the integrate kernel may raise it.  The
    // step ends an update period of the controlled cell when the iteration
    // count after it is a multiple of the period (the later kernels of the
    // step read the flag)
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.ctr->stall[parity] = 0;
        const CtrlConfig& c = *a.ctrl;
        a.ctr->measure = (c.active && (a.ctr->iter0 + a.ctr->steps_done + 1) % c.glob_update == 0) ? 1 : 0;
    }
    ContactPartial part = {0.0, 0.0, 0ull, 0ull, 0.0};
    bool unstable = false;
    // the measuring instantiation keeps what its terms need (force and
    // normal as stored, the branch length, k_n; zero for a pair not
    // touching) and forms the terms one at a time at the end
    double mf[3] = {0.0, 0.0, 0.0}, mn[3] = {0.0, 0.0, 0.0}, ml = 0.0, mkn = 0.0, mtouch = 0.0;
    if (k >= 0) {
        const gptr<const double4> xr = glb<const double4>(a.bod.xr);
        const gptr<const double4> vm = glb<const double4>(a.bod.vm);
        const gptr<const double4> wv = glb<const double4>(a.bod.w);
        const gptr<const uint16_t> mat = glb<const uint16_t>(a.bod.mat);
        const gptr<uint8_t> preal = glb(a.pr.real);
        using H = typename HistOf<PREC>::T;
        const gptr<H> hist = glb(reinterpret_cast<H*>(a.pr.h));
        const int s = BATCHED ? (int)glb<const uint16_t>(a.bod.scene)[sb] : 0;
        // an unbatched scene (periodic included) reads the descriptor's own
        // copy of its parameters: uniform, read-only here, so scalar loads
        const SceneParams& S = BATCHED ? a.scenes[s] : a.scene0;
        const double dt = S.dt;

        // #1's loads are issued without a branch, together with #2's: a
        // wall pair reads #2 in place of #1, a sphere pair reads wall 0 (the
        // wall table always holds at least one entry); the unused values are
        // then set aside
        const bool wall = sa < 0;
        const int32_t s1 = wall ? sb : sa;
        const double4 p2 = xr[sb];
        const double4 p1 = xr[s1];
        const int m2 = mat[sb];
        const int m1s = mat[s1];
        const Wall W = glb<const Wall>(a.walls)[wall ? -1 - sa : 0];
        const double x2 = p2.x, y2 = p2.y, z2 = p2.z, r2 = p2.w;
        const double x1 = wall ? 0.0 : p1.x, y1 = wall ? 0.0 : p1.y, z1 = wall ? 0.0 : p1.z;
        const double r1 = wall ? 0.0 : p1.w;
        const int m1 = wall ? W.mat : m1s;

        // ---- exact test, normal, overlap (always in double)
        bool real;
        bool in_box = false;       // a centre inside a box: overlap r + depth by definition
        double pen, inv_l = 0.0, l = 0.0;
        V3<double> n64;
        int cc[3] = {0, 0, 0};
        if (!wall) {
            if (PERIODIC) unpack_cell(pcell, cc);
            const SpherePairTest t =
                sphere_pair_test<PERIODIC>(x1, y1, z1, x2, y2, z2, r1, r2, S.H, cc[0], cc[1], cc[2]);
            real = t.real;
            l = sqrt(t.dd);
            inv_l = 1.0 / l;
            n64 = v3(t.dx * inv_l, t.dy * inv_l, t.dz * inv_l);
            pen = (r1 + r2) - l;
            if (pen < 0.0) pen = 0.0;
        } else if (!PRIMS || W.kind == kPlane) {
            const double xa = W.axis == 0 ? x2 : (W.axis == 1 ? y2 : z2);
            const double delta = xa - W.pos;
            real = fabs(delta) < r2;
            const double sg = W.sense != 0 ? (double)W.sense : (delta >= 0.0 ? 1.0 : -1.0);
            pen = r2 - sg * delta;
            n64 = v3(W.axis == 0 ? sg : 0.0, W.axis == 1 ? sg : 0.0, W.axis == 2 ? sg : 0.0);
        } else if constexpr (PRIMS) {
            // box (Ig2_Box_Sphere_ScGeom) or facet (Ig2_Facet_Sphere_ScGeom,
            // two-sided): normal from the closest point towards the centre
            const double xs[3] = {x2, y2, z2};
            double p[3];
            bool inside = false;
            if (W.kind == kBox)
                box_closest(W, xs, p, &inside);
            else
                facet_closest(W, xs, p);
            if (inside) {
                // the centre is in the box: out through the nearest face (first
                // of x-, x+, y-, y+, z-, z+ on a tie), overlap r + depth
                int ax = 0;
                double sgn = -1.0, depth = INFINITY;
                for (int q = 0; q < 3; ++q) {
                    const double dl = xs[q] - W.g[q], dh = W.g[3 + q] - xs[q];
                    if (dl < depth) {
                        depth = dl;
                        ax = q;
                        sgn = -1.0;
                    }
                    if (dh < depth) {
                        depth = dh;
                        ax = q;
                        sgn = 1.0;
                    }
                }
                real = true;
                in_box = true;
                pen = r2 + depth;
                n64 = v3(ax == 0 ? sgn : 0.0, ax == 1 ? sgn : 0.0, ax == 2 ? sgn : 0.0);
            } else {
                const double d0 = xs[0] - p[0], d1 = xs[1] - p[1], d2 = xs[2] - p[2];
                const double dist = sqrt((d0 * d0 + d1 * d1) + d2 * d2);
                real = dist < r2;
                pen = r2 - dist;
                if (dist > 0.0) {
                    n64 = v3(d0 / dist, d1 / dist, d2 / dist);
                } else {
                    // centre on the triangle: its face normal (v1 - v0) x (v2 - v0)
                    const V3<double> e1 = v3(W.g[3] - W.g[0], W.g[4] - W.g[1], W.g[5] - W.g[2]);
                    const V3<double> e2 = v3(W.g[6] - W.g[0], W.g[7] - W.g[1], W.g[8] - W.g[2]);
                    const V3<double> fn = cross(e1, e2);
                    const double len = sqrt(dot(fn, fn));
                    n64 = v3(fn.x / len, fn.y / len, fn.z / len);
                }
            }
        }

        if (!real) {
            // the contact is erased: drop its history (once), no force
            if (was_real) {
                hist[k] = H{};
                preal[k] = 0;
                set_row_bits(a, k, false);
            }
        } else {
            // ---- every load of a touching pair, issued together: both
            // bodies' velocities and spins, the history, the materials
            const double4 va = vm[s1], wa = wv[s1];
            const double4 vb = vm[sb], wb = wv[sb];
            const H hold = hist[k];
            const Material M1 = glb<const Material>(a.mats)[m1];
            const Material M2 = glb<const Material>(a.mats)[m2];
            const double tanphi64 = glb<const double>(a.tanphi)[m1 * a.nmat + m2];

            // ---- ScGeom inputs (a boundary's reference radius: the sphere's,
            // twice the sphere's for a facet)
            const double R1d = wall ? ((PRIMS && W.kind == kFacet) ? 2.0 * r2 : r2) : r1;
            const double R2d = r2;
            // a wall does not move
            const V3<double> v1d = wall ? v3(0.0, 0.0, 0.0) : v3(va.x, va.y, va.z);
            const V3<double> w1d = wall ? v3(0.0, 0.0, 0.0) : v3(wa.x, wa.y, wa.z);
            V3<double> v2d = v3(vb.x, vb.y, vb.z);
            const V3<double> w2d = v3(wb.x, wb.y, wb.z);
            if (PERIODIC) {
                // the image of #2 moves with the cell: (H - H_prev) c / dt
                // (one FP64 division, then three products)
                const double* D = S.dH;
                const double sx = (D[0] * (double)cc[0] + D[1] * (double)cc[1]) + D[2] * (double)cc[2];
                const double sy = (D[3] * (double)cc[0] + D[4] * (double)cc[1]) + D[5] * (double)cc[2];
                const double sz = (D[6] * (double)cc[0] + D[7] * (double)cc[1]) + D[8] * (double)cc[2];
                const double inv_dt = 1.0 / dt;
                v2d = v3(v2d.x + sx * inv_dt, v2d.y + sy * inv_dt, v2d.z + sz * inv_dt);
            }
            // relative translational velocity in double (difference of absolute values)
            const V3<double> dv64 = v2d - v1d;

            // ---- contact stiffnesses (and the visco-elastic dashpots)
            R kn, ks;
            double kn64 = 0.0, cn64 = 0.0, cs64 = 0.0;
            const bool ve = VISCEL && M2.viscel != 0;
            if (ve) {
                // Ip2_ViscElMat_ViscElMat_ViscElPhys: the pair's constants
                // scaled by the reduced mass; a body that cannot move (a
                // boundary, or a sphere with all six DOFs blocked) leaves the
                // other's own mass
                const gptr<const uint8_t> blk = glb<const uint8_t>(a.bod.blocked);
                const bool fixed1 = wall || blk[s1] == 63u, fixed2 = blk[sb] == 63u;
                const double m2m = sphere_mass(r2, M2.density);
                const double m1m = wall ? 0.0 : sphere_mass(r1, M1.density);
                double mr = m1m * m2m / (m1m + m2m);
                if (fixed1 && !fixed2) mr = m2m;
                if (fixed2 && !fixed1) mr = m1m;
                const ViscElPair P = glb<const ViscElPair>(a.ve)[m1 * a.nmat + m2];
                const double pi2 = 3.14159265358979323846 * 3.14159265358979323846;
                const double tc2 = P.tc * P.tc;
                kn64 = mr * (pi2 + P.len * P.len) / tc2;
                kn = (R)kn64;
                cn64 = -2.0 * mr * P.len / P.tc;
                ks = (R)(2.0 / 7.0 * mr * (pi2 + P.let * P.let) / tc2);
                cs64 = -2.0 / 7.0 * mr * P.let / P.tc;
            } else {
                // Ip2_FrictMat_FrictMat_FrictPhys: series springs k_i = E_i (2 R_i)
                const R k1 = (R)M1.young * ((R)2 * (R)R1d), k2 = (R)M2.young * ((R)2 * (R)R2d);
                kn = k1 * k2 / (k1 + k2);
                const R q1 = (R)M1.young_poisson * ((R)2 * (R)R1d), q2 = (R)M2.young_poisson * ((R)2 * (R)R2d);
                ks = q1 * q2 / (q1 + q2);
            }
            const R tanphi = (R)tanphi64;

            const V3<R> n = cvt<R>(n64);
            const R penr = (R)pen;
            const R Rd1 = (R)R1d, Rd2 = (R)R2d;
            const R dtr = (R)dt;

            // ---- shear update (section 2.1.3): both rotation increments from
            // the previous vector, then the sliding increment
            const V3<double> fs_old64 = v3(hold.fsx, hold.fsy, hold.fsz);
            const V3<R> fs_old = cvt<R>(fs_old64);
            const V3<R> nprev = v3((R)hold.nx, (R)hold.ny, (R)hold.nz);
            const V3<R> inc1 = cross(fs_old, cross(nprev, n));
            const V3<R> w1 = cvt<R>(w1d), w2 = cvt<R>(w2d);
            const R spin = (dtr / (R)2) * dot(n, w1 + w2);
            const V3<R> inc2 = cross(fs_old, spin * n);
            // v12 = alpha (v2 - v1) - (r2 w2 + r1 w1) x n, alpha = (r1 + r2)/l
            const R alpha = wall ? (R)1 : (R)((r1 + r2) * inv_l);
            const V3<R> rw = Rd2 * w2 + Rd1 * w1;
            const V3<R> v12 = alpha * cvt<R>(dv64) - cross(rw, n);
            const V3<R> vs = v12 - dot(n, v12) * n;
            const V3<R> dfs = ((v3<R>((R)0, (R)0, (R)0) - inc1) - inc2) - (ks * dtr) * vs;
            V3<double> fs64 = fs_old64 + cvt<double>(dfs);

            // ---- Law2_ScGeom_FrictPhys_CundallStrack; Law2_ScGeom_ViscElPhys_Basic
            // adds a normal dashpot on the overlap's rate -(v2 - v1).n (no
            // tension cut-off) and a shear dashpot that carries nothing while
            // the slider slides, the slider bounding the spring's part by
            // tan(phi) times the compressive normal force
            R fn_mag;
            double un = 0.0;
            if (ve) {
                // spring and dashpot in FP64 in both modes: near the end of a
                // contact they cancel, and k_n rounded to FP32 would leave its
                // rounding error against a small difference
                un = (n64.x * dv64.x + n64.y * dv64.y) + n64.z * dv64.z;
                fn_mag = (R)(kn64 * pen - cn64 * un);
            } else {
                fn_mag = kn * penr;
            }
            const R fmax = (ve && fn_mag < (R)0 ? (R)0 : fn_mag) * tanphi;
            const double fs_norm = sqrt(dot(fs64, fs64));
            const bool slide = fs_norm > (double)fmax;
            if (slide) {
                part.plast += (fs_norm - (double)fmax) * (double)fmax / (double)ks;
                const double ratio = (double)fmax / fs_norm;
                fs64 = ratio * fs64;
            }
            V3<R> fsr = cvt<R>(fs64);
            if (ve) {
                const V3<double> vs64 = cvt<double>(vs);
                const double vss = dot(vs64, vs64);
                if (!slide) fsr = cvt<R>(fs64 + (-cs64) * vs64);
                part.visc += ((cn64 * un) * un + (slide ? 0.0 : cs64 * vss)) * dt;
                part.el += 0.5 * ((kn64 * pen) * pen) + 0.5 * (dot(fs64, fs64) / (double)ks);
            } else {
                part.el += 0.5 * ((double)fn_mag * (double)fn_mag / (double)kn) + 0.5 * (dot(fs64, fs64) / (double)ks);
            }
            const V3<R> F = fn_mag * n + fsr;
            const V3<R> tau = cross(n, F);

            if constexpr (PREC == DEM_FP32_MIXED)
                hist[k] = H{fs64.x, fs64.y, fs64.z, pen, (float)n.x, (float)n.y, (float)n.z, (float)fn_mag};
            else
                hist[k] = H{fs64.x, fs64.y, fs64.z, pen, (double)n.x, (double)n.y, (double)n.z, (double)fn_mag};
            // the force record as three pairs (a record starts on an 8-byte
            // (FP32) or 16-byte (FP64) boundary of a 256-byte aligned array);
            // the FP64 linear law's integrate kernel reads the history instead
            if (PREC == DEM_FP32_MIXED) {
                const gptr<float2> q = glb(reinterpret_cast<float2*>(a.pr.frecf)) + 3 * (size_t)k;
                q[0] = make_float2((float)F.x, (float)F.y);
                q[1] = make_float2((float)F.z, (float)tau.x);
                q[2] = make_float2((float)tau.y, (float)tau.z);
            } else if (VISCEL) {
                const gptr<double2> q = glb(reinterpret_cast<double2*>(a.pr.frec)) + 3 * (size_t)k;
                q[0] = make_double2((double)F.x, (double)F.y);
                q[1] = make_double2((double)F.z, (double)tau.x);
                q[2] = make_double2((double)tau.y, (double)tau.z);
            }
            if (!was_real) {
                preal[k] = 1;
                set_row_bits(a, k, true);
            }
            if (wall)
                part.sw = 1;
            else
                part.ss = 1;
            const double rmin = wall ? r2 : (r1 < r2 ? r1 : r2);
            unstable = pen > rmin && !in_box;
            if constexpr (MEASURE) {
                mf[0] = (double)F.x;
                mf[1] = (double)F.y;
                mf[2] = (double)F.z;
                mtouch = 1.0;
                if (!wall) {
                    // sphere pairs only enter the stress and modulus terms
                    mn[0] = (double)n.x;
                    mn[1] = (double)n.y;
                    mn[2] = (double)n.z;
                    ml = l;
                    mkn = (double)kn;
                }
            }
        }
    }

    // ---- block slot: counts always (a wave counts its touching lanes with
    // one ballot), energies when tracked (fixed-order wave and block
    // combination, plain stores into this block's slot).  The largest
    // overlap is not reduced here: it is read from the history records on
    // request.
    __shared__ ContactPartial s_p[kMaxBlock / 64];
    __shared__ uint32_t s_bad[kMaxBlock / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    const bool energy = a.track_energy != 0;
    if (energy) {
        for (int off = 32; off > 0; off >>= 1) {
            part.el += __shfl_down(part.el, off, 64);
            part.plast += __shfl_down(part.plast, off, 64);
            if (VISCEL) part.visc += __shfl_down(part.visc, off, 64);
        }
    }
    part.ss = (unsigned long long)__popcll(__ballot(part.ss != 0ull));
    part.sw = (unsigned long long)__popcll(__ballot(part.sw != 0ull));
    const bool bad = __any(unstable);
    if (lane == 0) {
        s_p[wave] = part;
        s_bad[wave] = bad ? 1u : 0u;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double el = 0.0, pl = 0.0, vi = 0.0;
        unsigned long long ss = 0, sw = 0;
        uint32_t flags = 0;
        for (int w = 0; w < nwaves; ++w) {
            el += s_p[w].el;
            pl += s_p[w].plast;
            if (VISCEL) vi += s_p[w].visc;
            ss += s_p[w].ss;
            sw += s_p[w].sw;
            flags |= s_bad[w];
        }
        ContactAcc& acc = a.acc_contact[blockIdx.x];
        if (energy) {
            acc.el = el;
            acc.plast += pl;
            if (VISCEL) acc.visc += vi;
        }
        acc.ss = ss;
        acc.sw = sw;
        acc.ss_cum += ss;
        acc.sw_cum += sw;
        if (flags) a.ctr->unstable = 1;
    }
    if constexpr (MEASURE) {
        // the block's partial, one array per term (coalesced for the
        // reduction that follows the step): Love-Weber stress f_i (-l n_j)
        // (9), modulus k_n (l n_i n_i)^2 (3), |F| and the count
        __shared__ double s_net[kMaxBlock / 64][kNetworkWords];
        for (int q = 0; q < kNetworkWords; ++q) {
            double v;
            if (q < 9)
                v = mf[q / 3] * (-ml * mn[q % 3]);
            else if (q < 12) {
                const double dn = (ml * mn[q - 9]) * mn[q - 9];
                v = mkn * dn * dn;
            } else if (q == 12)
                v = sqrt(mf[0] * mf[0] + mf[1] * mf[1] + mf[2] * mf[2]);
            else
                v = mtouch;
            for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
            if (lane == 0) s_net[wave][q] = v;
        }
        __syncthreads();
        if (threadIdx.x < kNetworkWords) {
            double t = 0.0;
            for (int w = 0; w < nwaves; ++w) t += s_net[w][threadIdx.x];
            a.acc_ctrl[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = t;
        }
    }
}

template <int PREC, bool BATCHED, bool PERIODIC, bool MEASURE = false, bool PRIMS = false, bool VISCEL = false>
void launch_t(const StepArgs* args, int parity, int grid, int block, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1)
{
    const dim3 g(grid > 0 ? grid : 1), b(block);
    if (ev0)
        hipExtLaunchKernelGGL((k_contact<PREC, BATCHED, PERIODIC, MEASURE, PRIMS, VISCEL>), g, b, 0, st, ev0, ev1, 0,
                              args, parity);
    else
        hipLaunchKernelGGL((k_contact<PREC, BATCHED, PERIODIC, MEASURE, PRIMS, VISCEL>), g, b, 0, st, args, parity);
}

// the visco-elastic instantiation of a scene kind: boundaries of every kind
// when aperiodic
template <int PREC>
void launch_viscel(const StepArgs* args, int parity, int grid, int block, hipStream_t st, hipEvent_t ev0,
                   hipEvent_t ev1, bool batched, bool periodic)
{
    if (periodic)
        launch_t<PREC, false, true, false, false, true>(args, parity, grid, block, st, ev0, ev1);
    else if (batched)
        launch_t<PREC, true, false, false, true, true>(args, parity, grid, block, st, ev0, ev1);
    else
        launch_t<PREC, false, false, false, true, true>(args, parity, grid, block, st, ev0, ev1);
}

}  // namespace

void launch_contact(const StepArgs* args, int parity, int grid, int precision, bool batched, bool periodic,
                    int block, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1, bool measure, bool prims, bool viscel)
{
    if (viscel) {
        if (precision == DEM_FP32_MIXED)
            launch_viscel<DEM_FP32_MIXED>(args, parity, grid, block, st, ev0, ev1, batched, periodic);
        else
            launch_viscel<DEM_FP64>(args, parity, grid, block, st, ev0, ev1, batched, periodic);
        return;
    }
    if (prims && !periodic) {
        if (precision == DEM_FP32_MIXED) {
            if (batched) launch_t<DEM_FP32_MIXED, true, false, false, true>(args, parity, grid, block, st, ev0, ev1);
            else launch_t<DEM_FP32_MIXED, false, false, false, true>(args, parity, grid, block, st, ev0, ev1);
        } else {
            if (batched) launch_t<DEM_FP64, true, false, false, true>(args, parity, grid, block, st, ev0, ev1);
            else launch_t<DEM_FP64, false, false, false, true>(args, parity, grid, block, st, ev0, ev1);
        }
        return;
    }
    if (measure && periodic && !batched) {
        if (precision == DEM_FP32_MIXED) launch_t<DEM_FP32_MIXED, false, true, true>(args, parity, grid, block, st, ev0, ev1);
        else launch_t<DEM_FP64, false, true, true>(args, parity, grid, block, st, ev0, ev1);
        return;
    }
    if (precision == DEM_FP32_MIXED) {
        if (batched) launch_t<DEM_FP32_MIXED, true, false>(args, parity, grid, block, st, ev0, ev1);
        else if (periodic) launch_t<DEM_FP32_MIXED, false, true>(args, parity, grid, block, st, ev0, ev1);
        else launch_t<DEM_FP32_MIXED, false, false>(args, parity, grid, block, st, ev0, ev1);
    } else {
        if (batched) launch_t<DEM_FP64, true, false>(args, parity, grid, block, st, ev0, ev1);
        else if (periodic) launch_t<DEM_FP64, false, true>(args, parity, grid, block, st, ev0, ev1);
        else launch_t<DEM_FP64, false, false>(args, parity, grid, block, st, ev0, ev1);
    }
}

}  // namespace dem
