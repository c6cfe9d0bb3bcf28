// dem_internal.hpp -- device data layout and kernel launchers shared by the
// runtime (runtime.cpp) and the kernel sources (*.hip) of libdem_hip.so.
//
// Layout (all structure-of-arrays, bodies in cell (Morton) order, 256-byte
// aligned): one "slot" per sphere, reordered at every broad-phase run; the
// id <-> slot maps let the ABI speak ids.  Candidate pairs are stored once
// (owner = #1 of the contact); each body keeps a row of its candidate pairs
// sorted by partner id, which fixes the order of its force sum.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <cstdint>
#include <type_traits>

#include "dem.h"

namespace dem {

constexpr int kMaxWallsPerScene = 64;   // fixed boundaries (planes, boxes, facets) per scene
// A row entry: the pair's index, the body's side and whether the pair
// touched at its last evaluation (kept current by the contact kernel, so
// that a body's force sum reads no flag of its own).
constexpr uint32_t kNegSign = 0x80000000u;  // body is #1, adds -F
constexpr uint32_t kRealBit = 0x40000000u;  // the pair touches
constexpr uint32_t kPairMask = 0x3fffffffu;

// Per-scene parameters, read by the kernels through the body's scene index.
struct SceneParams {
    double dt;
    double gravity[3];
    double damping;
    int32_t damp_rot;
    int32_t homo_deform;
    double verlet;            // Delta L
    int32_t wall_begin;       // into the global wall table
    int32_t wall_count;
    // broad-phase grid (rewritten at every run)
    double origin[3];         // aperiodic: lower corner
    double inv_h[3];          // cells per metre (aperiodic) or cells per unit of fractional coordinate
    int32_t dims[3];
    int32_t cell_offset;      // first cell of this scene in the cell table
    // periodic cell
    int32_t periodic;
    int32_t pad_;
    double H[9];              // current cell
    double Hinv[9];
    double dH[9];             // H - H_prev: the image shift moved by dH c over the last step
    double L[9];              // velGrad
    double Lprev[9];          // velGrad of the previous step
    double trsf[9];           // accumulated cell transformation
    double verlet_cell_rate;  // 1/2 |L|_F (2 r_max + 4 Delta L): Verlet budget used per unit time by the mean field
    double rmax;              // largest radius of the scene at the run
    double cellw[3];          // metric width of a grid cell along each axis (>= the cell size h)
    // Two-level grid for wide size ratios: every sphere is binned on the
    // grid above (level 0, cells >= 2 r_split + 2 Delta L; this also fixes
    // the bodies' memory order), and the spheres of radius > r_split also on
    // a coarse grid of their own (level 1, cells >= 2 r_max + 2 Delta L,
    // an index array of their slots).  A sphere finds its partners of radius
    // <= r_split on level 0 and the larger ones on level 1.  r_split = 0: one
    // level (cells >= 2 r_max + 2 Delta L).
    double r_split;
    double origin2[3];
    double inv_h2[3];
    double cellw2[3];
    int32_t dims2[3];
    int32_t cell_offset2;
};

// A fixed boundary: an infinite axis-aligned plane (utils.wall: axis,
// sense, pos), an axis-aligned box (Box: g = lo[3], hi[3]) or a triangle
// (Facet: g = v0, v1, v2).  It is #1 of its contacts.
enum BoundaryKind : int32_t { kPlane = 0, kBox = 1, kFacet = 2 };
struct Wall {
    int32_t axis;
    int32_t sense;
    int32_t mat;
    int32_t id;
    double pos;
    int32_t kind;
    int32_t pad_;
    double g[9];
};

// Closest point of a box or a triangle to x (device code of the broad phase
// and the contact kernel).  Box: the clamp of x to [lo, hi]; `inside` when x
// is in the box.  Triangle: the region test over vertices, edges and face
// by the signs of the barycentric quantities (Ericson, Real-Time Collision
// Detection, section 5.1.5).
__device__ inline void box_closest(const Wall& W, const double* x, double* p, bool* inside)
{
    bool in = true;
    for (int k = 0; k < 3; ++k) {
        const double lo = W.g[k], hi = W.g[3 + k];
        p[k] = x[k] < lo ? lo : (x[k] > hi ? hi : x[k]);
        if (x[k] < lo || x[k] > hi) in = false;
    }
    *inside = in;
}

__device__ inline void facet_closest(const Wall& W, const double* x, double* p)
{
    const double* a = &W.g[0];
    const double* b = &W.g[3];
    const double* c = &W.g[6];
    double ab[3], ac[3], ap[3];
    for (int k = 0; k < 3; ++k) {
        ab[k] = b[k] - a[k];
        ac[k] = c[k] - a[k];
        ap[k] = x[k] - a[k];
    }
    auto dot = [](const double* u, const double* v) { return (u[0] * v[0] + u[1] * v[1]) + u[2] * v[2]; };
    const double d1 = dot(ab, ap), d2 = dot(ac, ap);
    if (d1 <= 0.0 && d2 <= 0.0) {
        for (int k = 0; k < 3; ++k) p[k] = a[k];
        return;
    }
    double bp[3];
    for (int k = 0; k < 3; ++k) bp[k] = x[k] - b[k];
    const double d3 = dot(ab, bp), d4 = dot(ac, bp);
    if (d3 >= 0.0 && d4 <= d3) {
        for (int k = 0; k < 3; ++k) p[k] = b[k];
        return;
    }
    const double vc = d1 * d4 - d3 * d2;
    if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) {
        const double t = d1 / (d1 - d3);
        for (int k = 0; k < 3; ++k) p[k] = a[k] + t * ab[k];
        return;
    }
    double cp[3];
    for (int k = 0; k < 3; ++k) cp[k] = x[k] - c[k];
    const double d5 = dot(ab, cp), d6 = dot(ac, cp);
    if (d6 >= 0.0 && d5 <= d6) {
        for (int k = 0; k < 3; ++k) p[k] = c[k];
        return;
    }
    const double vb = d5 * d2 - d1 * d6;
    if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) {
        const double t = d2 / (d2 - d6);
        for (int k = 0; k < 3; ++k) p[k] = a[k] + t * ac[k];
        return;
    }
    const double va = d3 * d6 - d5 * d4;
    if (va <= 0.0 && (d4 - d3) >= 0.0 && (d5 - d6) >= 0.0) {
        const double t = (d4 - d3) / ((d4 - d3) + (d5 - d6));
        for (int k = 0; k < 3; ++k) p[k] = b[k] + t * (c[k] - b[k]);
        return;
    }
    const double den = 1.0 / ((va + vb) + vc);
    const double v = vb * den, w = vc * den;
    for (int k = 0; k < 3; ++k) p[k] = (a[k] + ab[k] * v) + ac[k] * w;
}

// Distance from x to a box or triangle (0 inside a box): the broad phase's
// candidate test against a boundary.
__device__ inline double boundary_distance(const Wall& W, const double* x)
{
    double p[3];
    if (W.kind == kBox) {
        bool inside;
        box_closest(W, x, p, &inside);
        if (inside) return 0.0;
    } else {
        facet_closest(W, x, p);
    }
    const double d0 = x[0] - p[0], d1 = x[1] - p[1], d2 = x[2] - p[2];
    return sqrt((d0 * d0 + d1 * d1) + d2 * d2);
}

// Material constants as the kernels need them.
struct Material {
    double young;
    double young_poisson;     // E * nu
    double density;
    int32_t viscel;           // 1: ViscElMat (visco-elastic law), 0: FrictMat
    int32_t pad_;
};

// Pair constants of the visco-elastic law (Ip2_ViscElMat_ViscElMat_ViscElPhys
// from contact time and restitution coefficients): the means of the two
// materials' tc, and ln of the means of their en and et.  The coefficients
// follow per contact from the reduced mass m:
//   kn = m (pi^2 + len^2)/tc^2, cn = -2 m len/tc,
//   ks = 2/7 m (pi^2 + let^2)/tc^2, cs = -2/7 m let/tc.
struct ViscElPair {
    double tc, len, let, pad_;
};

// Body arrays of one buffer set.  The per-body vectors are packed four
// doubles wide (32 bytes, one aligned load), so that gathering a partner's
// position and radius, or its velocity, touches one memory segment.
struct Bodies {
    double4 *xr;              // x, y, z, radius
    double4 *vm;              // vx, vy, vz, and the Verlet account: non-affine displacement
                              // accumulated since the last broad-phase run
    double4 *w;               // wx, wy, wz, 0
    double4 *q;               // qw, qx, qy, qz
    uint16_t *mat;            // material index
    uint8_t *blocked;
    int32_t *id;              // slot -> body id
    uint16_t *scene;          // slot -> scene (batched only)
    int32_t *period;          // periodic: packed integer period of the body at the last run
};

// A sphere's mass, m = 4/3 pi r^3 rho, computed where it is needed (it is
// not stored: the fourth word of vm carries the Verlet account), in the
// same order of operations and without contraction, as the host computes
// it when the sphere is added.
__device__ inline double sphere_mass(double r, double rho)
{
#pragma clang fp contract(off)
    return 4.0 / 3.0 * 3.14159265358979323846 * r * r * r * rho;
}

// A pair's history record (64 bytes, one aligned segment): the shear force
// on #2 after the Coulomb cap, the normal, the overlap and the normal force
// of its last evaluation; a zero normal marks a pair that did not touch.
// Under the linear law in FP64 the record is also the pair's force record:
// the force on #2 is fn n + Fs and its torque term n x (fn n + Fs), so no
// separate force record is written (one 64-byte segment per gather).
struct HistRec {
    double fsx, fsy, fsz;     // shear force (the spring's part under the visco-elastic law)
    double pen;               // overlap of the last evaluation
    double nx, ny, nz;
    double fn;                // signed normal force on #2 along n: k_n pen (linear law), k_n pen - c_n u_n (visco-elastic)
};

// The FP32-mixed history record (48 bytes): the shear force and the overlap
// in FP64 as in FP64 mode, the normal and the normal force in FP32 (their
// precision in this mode, so nothing is lost by storing them narrower).
struct HistRec32 {
    double fsx, fsy, fsz;
    double pen;
    float nx, ny, nz;
    float fn;
};
static_assert(sizeof(HistRec) == 64 && sizeof(HistRec32) == 48, "history record sizes");
template <int PREC>
struct HistOf {
    using T = HistRec;
};
template <>
struct HistOf<DEM_FP32_MIXED> {
    using T = HistRec32;
};
inline size_t hist_bytes(int precision) { return precision == DEM_FP32_MIXED ? sizeof(HistRec32) : sizeof(HistRec); }
__host__ __device__ inline HistRec widen(const HistRec& h) { return h; }
__host__ __device__ inline HistRec widen(const HistRec32& h)
{
    return HistRec{h.fsx, h.fsy, h.fsz, h.pen, (double)h.nx, (double)h.ny, (double)h.nz, (double)h.fn};
}
// record k of a history array of the precision's layout, widened
template <int PREC>
__device__ inline HistRec hist_load(const HistRec* base, size_t k)
{
    return widen(reinterpret_cast<const typename HistOf<PREC>::T*>(base)[k]);
}

// Candidate pairs after a broad-phase run, the pairs that touched at the
// last evaluation first (a stable partition of the owner-sorted order), so
// that the contact kernel's touching pairs, their history and force records
// are dense in memory and its waves rarely mix the two paths.
struct Pairs {
    int32_t *a;               // slot of #1, or -1 - wall index
    int32_t *b;               // slot of #2
    int32_t *cell;            // packed image of #2 (periodic), 0 otherwise
    int32_t *pid;             // id of the non-owner partner (for history carry-over)
    uint8_t *real;            // 1 when the pair touched at the last evaluation
    int32_t *ea;              // index of the pair's entry in #1's row (-1: #1 is a boundary)
    int32_t *eb;              // index of the pair's entry in #2's row
    HistRec *h;               // history (HistRec32 records in FP32-mixed mode: see HistOf)
    // force on #2 and n x F of the last step, one record of kForceWords
    // values per pair (one contiguous gather per real row entry); written
    // only where the history record is not enough (see uses_force_records)
    double *frec;             // FP64 mode (visco-elastic law)
    float *frecf;             // FP32-mixed mode
};
constexpr int kForceWords = 6;

// Where the integrate kernel and the reports take a pair's force from: a
// force record (FP32-mixed: 24 bytes, smaller than the history record;
// the visco-elastic law: its shear dashpot is not in the history), or the
// history record itself (FP64 linear law).
inline bool uses_force_records(int precision, bool viscel) { return precision == DEM_FP32_MIXED || viscel; }

// Rows: for every slot, its candidate pairs sorted by partner id.
struct Rows {
    int32_t *start;           // nslots + 1
    uint32_t *ent;            // pair index | kNegSign when the body is #1
};

// History of the previous candidate list, keyed by ids: per owner id a
// range of the owner-sorted ("canonical") order with each pair's partner id
// and image, and where that pair sits in the partitioned arrays.
struct History {
    int32_t *own_begin;       // by body id
    int32_t *own_count;
    int32_t *pid;             // canonical: partner id
    int32_t *cell;            // canonical: image
    int32_t *map;             // canonical -> index of the pair in the partitioned arrays
    const HistRec *h;         // partitioned order
};

// Device-side flags and counters (one struct in device memory).  The hot
// kernels use no atomics: flags are plain stores of 1, the step counter has
// a single writer, and energies / contact counts go to per-block slots.
struct Counters {
    int32_t stall[2];               // by step parity: a broad-phase run is needed before the next step
    int32_t steps_done;             // steps completed since the host last reset it (block 0 of integrate)
    int32_t halt;                   // the controlled cell reached its goal: the launch chain stops
    int64_t iter0;                  // the scene's iteration count when the host last reset steps_done
    int32_t nonfinite;              // a NaN/Inf position or velocity appeared
    int32_t unstable;               // an overlap exceeded a radius
    double verlet_limit;            // per-body displacement budget (0.98 Delta L)
    double verlet_cell_step;        // mean-field share of the budget used per step (periodic)
    int32_t measure;                // this step ends an update period of the controlled cell (set by contact)
    int32_t pad_;
};

// The stress/strain-controlled periodic cell (PeriTriaxController driven by
// the packing stiffness), run on the device after the steps that make the
// iteration count a multiple of glob_update.
// iso: the isotropic compressor (PeriIsoCompressor with keepProportions):
// the goals are series[0 .. n_series), one after another, controlled on the
// mean stress with one rate for all axes; stress_mask and goal are unused.
constexpr int kMaxStressSeries = 8;
struct CtrlConfig {
    double goal[3];
    int32_t stress_mask;
    int32_t glob_update;
    double max_rate[3];
    double grow_damping;
    double max_unbalanced;
    double abs_tol;
    double rel_tol;
    int32_t stop_when_done;
    int32_t active;
    int32_t iso;
    int32_t n_series;
    double series[kMaxStressSeries];
};
struct CtrlState {
    double stress[3], strain[3], rate[3], stiff[3];
    double unbalanced;
    int64_t updates;
    int32_t done;
    int32_t series_index;     // iso: the goal being driven to
};
// The controlled cell's sums come from the step kernels' own blocks on its
// update steps: the contact kernel's measuring instantiation (kNetworkWords
// per block in acc_ctrl, stored term-major: term q of block b at
// q * nblocks_contact + b) and the integrate kernel's slots (IntAcc.fsum /
// fcnt).  A first reduction level (kCtrlReduceGrid blocks, update steps
// only) brings them to kCtrlReduceGrid partials in acc_ctrl2 for the
// cell-update block.
constexpr int kCtrlReduceGrid = 256;

// Per-block slots of the contact kernel: the last step's values and the
// running sums since the host last folded them (fixed block order).
struct ContactAcc {
    double el;                      // elastic energy of the block's contacts, last step
    double plast;                   // plastic work, cumulative
    unsigned long long ss, sw;      // real contacts of the last step
    unsigned long long ss_cum, sw_cum;
    double visc;                    // dashpot work of the visco-elastic law, cumulative
};

// Per-block slots of the integrate kernel.
struct IntAcc {
    double kin, rot;                // last step
    double grav, damp;              // cumulative
    double fsum, fcnt;              // |resultant contact force| over dynamic spheres and their number,
                                    // at the last step that ended an update period of the controlled cell
};

struct StepArgs {
    Bodies bod;
    Pairs pr;
    Rows rows;
    const Wall* walls;
    const Material* mats;
    const double* tanphi;           // nmat x nmat, tan(min(phi1, phi2))
    const ViscElPair* ve;           // nmat x nmat, visco-elastic pair constants
    int32_t nmat;
    SceneParams* scenes;            // device table (k_cell_update keeps a periodic cell's entry current)
    SceneParams scene0;             // copy of scene 0 for unbatched kernels
    int32_t nscenes;
    int32_t nslots;
    int32_t npairs;
    Counters* ctr;
    ContactAcc* acc_contact;        // one slot per contact block
    IntAcc* acc_integrate;          // one slot per integrate block
    int32_t track_energy;
    // stress/strain-controlled cell (periodic, unbatched): configuration,
    // state, and the contact kernel's per-block sums on update steps
    const CtrlConfig* ctrl;
    CtrlState* ctrl_state;
    double* acc_ctrl;
    double* acc_ctrl2;              // kCtrlReduceGrid x (kNetworkWords + 2)
    int32_t nblocks_contact;        // blocks of the contact kernel (its grid)
    int32_t nblocks_integrate;      // slots of acc_integrate written by the integrate kernel
    int32_t use_frec;               // forces come from the force records (uses_force_records), else the history
    int32_t pad_;
};

// Global-memory view of a buffer pointer.  The step kernels load their
// pointers from a device descriptor, so the compiler cannot prove that they
// address global memory and would emit flat loads and stores (64-bit
// addresses, waits shared with LDS and scalar loads); the cast lets it emit
// global ones.  Only meaningful in device code (the host pass, which checks
// the kernels' source, sees plain pointers).
#if defined(__HIP_DEVICE_COMPILE__)
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
#else
template <typename T>
using gptr = T*;
#endif
template <typename T>
__device__ inline gptr<T> glb(T* p)
{
    return (gptr<T>)p;
}

// ---------------------------------------------------------------- launchers
// (defined in the .hip files; all asynchronous on `st`)

// prim.hip
size_t scan_temp_bytes(int n);
void exclusive_scan_u32(const uint32_t* in, uint32_t* out, int n, void* temp, uint32_t* total_dev,
                        hipStream_t st);
size_t radix_temp_bytes(int n);
void radix_sort_pairs(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt, uint32_t* vals_alt, int n,
                      int nbits, void* temp, hipStream_t st, bool* result_in_alt);

// broadphase.hip
struct GridArgs {
    Bodies bod;
    const SceneParams* scenes;
    SceneParams scene0;
    int32_t nscenes;
    int32_t nslots;
    int32_t scene_bits;        // bits of the scene index in the key
    int32_t morton_bits;       // bits per axis
    int32_t* period_range;     // set to 1 by k_keys when a body's period is outside [-512, 511]
    const uint32_t* large_slot;  // level 1: slots of the spheres above r_split, in coarse-cell order (or null)
};
size_t bounds_temp_bytes(int nslots);
void launch_bounds(const Bodies& b, int nslots, int nscenes, double* out6, void* temp, hipStream_t st);
void launch_keys(const GridArgs& g, uint64_t* keys, uint32_t* vals, hipStream_t st);
void launch_permute(const Bodies& src, const Bodies& dst, const uint32_t* order, int nslots, bool batched,
                    bool periodic, int32_t* slot_of_id, hipStream_t st);
void launch_cells(const GridArgs& g, const uint64_t* sorted_keys, uint32_t* cell_start, uint32_t* cell_end,
                  int ncells, hipStream_t st);
// Level 1 of a two-level grid: flags of the spheres above their scene's
// r_split (then scanned by the caller), their coarse-cell keys and slots at
// the scanned positions, and (after sorting those) the level's cell ranges
// into the sorted index array.
void launch_large_flags(const GridArgs& g, uint32_t* flag, hipStream_t st);
void launch_large_keys(const GridArgs& g, const uint32_t* scan, uint64_t* keys2, uint32_t* vals2, hipStream_t st);
void launch_cells_large(const GridArgs& g, const uint64_t* sorted_keys2, int nlarge, uint32_t* cell_start,
                        uint32_t* cell_end, int ncells, hipStream_t st);
struct SweepArgs {
    GridArgs g;
    const uint32_t* cell_start;
    const uint32_t* cell_end;
    const Wall* walls;
    uint32_t* count;           // per slot: the count pass's counts, then how the fill left each row
    const int32_t* row_start;  // fill pass
    // the fill pass writes each row sorted by (partner id, image) into ent_*
    // where the row fits its block's LDS pool, else in the order found
    // (raw_*), which the rank passes sort into ent_*; every entry's row goes
    // to ent_body, and ent_own marks the entries that own their pair
    int32_t* raw_slot;         // partner slot or -1 - wall
    int32_t* raw_pid;          // partner id
    int32_t* raw_cell;         // packed image shift of the partner
    int32_t* ent_body;         // slot whose row holds the entry
    int32_t* ent_slot;
    int32_t* ent_pid;
    int32_t* ent_cell;
    uint32_t* ent_own;         // 1 when this entry owns the pair
    int32_t max_row;
    int32_t nent;
    int32_t nlarge;            // spheres on level 1 (their sweeps run as a pass of their own)
};
void launch_sweep_count(const SweepArgs& a, hipStream_t st);
void launch_sweep_fill(const SweepArgs& a, hipStream_t st);  // fill, then the rank pass
struct PairBuildArgs {
    Bodies bod;
    const int32_t* row_start;
    const int32_t* ent_slot;
    const int32_t* ent_pid;
    const int32_t* ent_cell;
    const uint32_t* own_scan;  // exclusive scan of the owner flags
    const uint32_t* ent_own;
    const int32_t* ent_body;   // slot whose row holds the entry
    Rows rows;
    Pairs pr;                  // the new list (partitioned order)
    History hist_new;          // own ranges and canonical arrays of the new list
    History hist_old;          // previous list
    int32_t* ca;               // canonical #1 / #2 slots (scratch)
    int32_t* cb;
    int32_t* found;            // canonical: index of the pair in the previous list's arrays, -1 if new
    uint32_t* flag;            // canonical: 1 when the carried history says the pair touched (+1 entry, 0)
    uint32_t* flag_scan;       // exclusive scan of flag; flag_scan[npairs] = number of touching pairs
    int32_t nslots;
    int32_t nent;
    int32_t npairs;
    int32_t has_old;
    int32_t hist_f32;          // history records are HistRec32 (FP32-mixed)
};
// canonical pair arrays and rows (pair_build), history lookup (carry_find),
// then, after the host scans `flag`, the partition into the final arrays
// and the rows' entries renumbered to it (partition)
void launch_pair_build(const PairBuildArgs& a, hipStream_t st);
void launch_carry_find(const PairBuildArgs& a, hipStream_t st, int old_nbodies);
void launch_partition(const PairBuildArgs& a, hipStream_t st);

// contact.hip
// ev0/ev1 (optional): events stamped at the kernel's own start and end
// (hipExtLaunchKernelGGL), used by the timing mode.
// measure: the step ends an update period of the controlled cell (periodic,
// unbatched): the measuring instantiation runs (the host decides per step;
// captured graphs are keyed by the period's phase at their first step)
// prims: the world holds a box or a facet (aperiodic): the instantiation
// with their geometry runs; viscel: the world holds visco-elastic materials
// (their instantiation, which takes every boundary kind, runs)
void launch_contact(const StepArgs* args, int parity, int grid, int precision, bool batched, bool periodic,
                    int block, hipStream_t st, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr,
                    bool measure = false, bool prims = false, bool viscel = false);

// integrate.hip
// frec: uses_force_records(precision, world has visco-elastic materials)
void launch_integrate(const StepArgs* args, int parity, int grid, int precision, bool batched, bool periodic,
                      bool frec, int block, hipStream_t st, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// One block after the step: the periodic cell's update, then (when the
// controlled cell is on and the step is one of its updates) the
// controller, from the contact and integrate kernels' partial sums.
void launch_cell_update(const StepArgs* args, int parity, hipStream_t st);
// largest Verlet account over the bodies, as the bits of a double, into
// *out (which the caller zeroes)
void launch_max_account(const Bodies& b, int n, unsigned long long* out, hipStream_t st);
// first reduction level of the controller's partial sums (update steps only)
void launch_ctrl_reduce(const StepArgs* args, int parity, hipStream_t st);
void launch_body_forces(const StepArgs& a, int precision, double* f3, double* t3, hipStream_t st);
// Sums over the last step's real contacts, kNetworkWords doubles per block
// (stress.hip): Love-Weber stress (9), modulus of the normal springs per
// axis (3), sum of |F| and count (2); `scene` selects a batch scene.
constexpr int kNetworkWords = 14;
int stress_blocks(int npairs);
// Largest overlap / smaller radius (a boundary's sphere's radius) over the
// pairs that touched at the last step, from their history records, as the
// bits of a non-negative double into *out (which the caller zeroes).
void launch_max_overlap(const StepArgs& a, int precision, unsigned long long* out, hipStream_t st);
// Force on #2 of every pair (3 doubles per pair; 0 for a pair not touching).
void launch_pair_forces(const StepArgs& a, int precision, double* f3, hipStream_t st);
void launch_network(const StepArgs& a, int precision, bool batched, int scene, double* part, hipStream_t st);
// The Love-Weber stress sums (9 doubles, times the volume) of one scene
// computed in the library's fixed device scratch, allocating nothing; returns
// the device address of the nine words (valid until the next such call on
// this GPU), or nullptr when the scratch is unavailable or the pair count is
// 0 or above stress_noalloc_max_pairs().
constexpr int kNoAllocMaxPerThread = 256;
int64_t stress_noalloc_max_pairs();
const double* launch_stress_noalloc(const StepArgs& a, int precision, bool batched, int scene, hipStream_t st);
// Sums over the bodies of one scene, kBodyWords doubles per block
// (integrate.hip): sum and largest |resultant contact force| over the
// dynamic spheres, their number, and the smallest stiffness-based critical
// timestep (eqs. 2.12-2.14; +inf without contacts).
constexpr int kBodyWords = 4;
int body_blocks(int nslots);
void launch_body_measures(const StepArgs& a, int precision, bool batched, int scene, double* part, hipStream_t st);


}  // namespace dem
