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
#include <cstdint>
#include <type_traits>

#include "dem.h"

namespace dem {

constexpr int kMaxWallsPerScene = 16;
constexpr uint32_t kNegSign = 0x80000000u;  // row entry: body is #1, adds -F
constexpr uint32_t kPairMask = 0x7fffffffu;

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
};

struct Wall {
    int32_t axis;
    int32_t sense;
    int32_t mat;
    int32_t id;
    double pos;
};

// Material constants as the kernels need them.
struct Material {
    double young;
    double young_poisson;     // E * nu
    double density;
};

// Body arrays of one buffer set.
struct Bodies {
    double *x, *y, *z;
    double *vx, *vy, *vz;
    double *wx, *wy, *wz;
    double *qw, *qx, *qy, *qz;
    double *rad, *mass;
    uint8_t *mat;
    uint8_t *blocked;
    int32_t *id;              // slot -> body id
    uint16_t *scene;          // slot -> scene (batched only)
    int32_t *period;          // periodic: packed integer period of the body at the last run
};

// Candidate pairs after a broad-phase run.
struct Pairs {
    int32_t *a;               // slot of #1, or -1 - wall index
    int32_t *b;               // slot of #2
    int32_t *cell;            // packed image of #2 (periodic), 0 otherwise
    int32_t *pid;             // id of the non-owner partner (for history carry-over)
    double *fsx, *fsy, *fsz;  // shear force on #2 (history)
    double *nx, *ny, *nz;     // normal of the last step; 0 for a non-real pair
    double *fx, *fy, *fz;     // total force on #2 of the last step
    double *tx, *ty, *tz;     // n x F of the last step (torque = -r_k * this)
    float *fxf, *fyf, *fzf;   // FP32-mixed mode per-pair force
    float *txf, *tyf, *tzf;
};

// Rows: for every slot, its candidate pairs sorted by partner id.
struct Rows {
    int32_t *start;           // nslots + 1
    uint32_t *ent;            // pair index | kNegSign when the body is #1
};

// History of the previous candidate list, keyed by ids.
struct History {
    int32_t *own_begin;       // by body id
    int32_t *own_count;
    int32_t *pid;             // by pair: partner id
    int32_t *cell;
    double *fsx, *fsy, *fsz, *nx, *ny, *nz;
};

// Device-side counters and accumulators (one struct in device memory).
struct Counters {
    unsigned long long vmax_bits;   // this step: max over bodies of the non-affine displacement (double bits)
    double verlet_acc;              // displacement bound accumulated since the last broad-phase run
    double verlet_limit;            // a run is needed once verlet_acc exceeds this
    double verlet_cell_step;        // mean-field term added every step (periodic)
    int32_t stall;                  // 1: a broad-phase run is needed before the next step
    int32_t steps_done;             // steps completed since the host last reset it
    int32_t nonfinite;              // a NaN/Inf position or velocity appeared
    int32_t unstable;               // an overlap exceeded a radius
    unsigned int blocks_done_contact;
    unsigned int blocks_done_integrate;
    unsigned long long cur_ss, cur_sw;    // real contacts counted during this step
    unsigned long long last_ss, last_sw;  // real contacts of the last completed step
    unsigned long long contact_steps;     // sum over completed steps
    double e_kin, e_rot, e_el, e_grav, e_damp, e_plast;
};

// Energy / count partials of one block.
struct BlockPartial {
    double e[4];                    // contact: el, plast, -, -   integrate: kin, rot, grav, damp
    unsigned long long n[2];        // contact: ss, sw
    double vmax;
    double pad_;
};

struct StepArgs {
    Bodies bod;
    Pairs pr;
    Rows rows;
    const Wall* walls;
    const Material* mats;
    const double* tanphi;           // nmat x nmat, tan(min(phi1, phi2))
    int32_t nmat;
    SceneParams* scenes;            // device table (the last integrate block updates a periodic cell)
    SceneParams scene0;             // copy of scene 0 for unbatched kernels
    int32_t nscenes;
    int32_t nslots;
    int32_t npairs;
    Counters* ctr;
    BlockPartial* part_contact;
    BlockPartial* part_integrate;
    int32_t track_energy;
};

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
};
void launch_bounds(const Bodies& b, const uint16_t* scene, int nslots, int nscenes, double* out6,
                   hipStream_t st);
void launch_keys(const GridArgs& g, uint64_t* keys, uint32_t* vals, hipStream_t st);
void launch_permute(const Bodies& src, const Bodies& dst, const uint32_t* order, int nslots, bool batched,
                    bool periodic, int32_t* slot_of_id, hipStream_t st);
void launch_cells(const GridArgs& g, const uint64_t* sorted_keys, uint32_t* cell_start, uint32_t* cell_end,
                  int ncells, hipStream_t st);
struct SweepArgs {
    GridArgs g;
    const uint32_t* cell_start;
    const uint32_t* cell_end;
    const Wall* walls;
    uint32_t* count;           // per slot
    const int32_t* row_start;  // fill pass
    int32_t* ent_slot;         // fill pass: partner slot or -1 - wall
    int32_t* ent_pid;          // partner id
    int32_t* ent_cell;         // packed image shift of the partner
    uint32_t* ent_own;         // 1 when this entry owns the pair
    int32_t max_row;
};
void launch_sweep_count(const SweepArgs& a, hipStream_t st);
void launch_sweep_fill(const SweepArgs& a, hipStream_t st);
struct PairBuildArgs {
    Bodies bod;
    const int32_t* row_start;
    const int32_t* ent_slot;
    const int32_t* ent_pid;
    const int32_t* ent_cell;
    const uint32_t* own_scan;  // exclusive scan of the owner flags
    const uint32_t* ent_own;
    Rows rows;
    Pairs pr;
    History hist_new;          // own ranges of the new list (by id)
    History hist_old;          // previous list
    int32_t nslots;
    int32_t nent;
    int32_t npairs;
    int32_t has_old;
};
void launch_pair_build(const PairBuildArgs& a, hipStream_t st);
void launch_carry_over(const PairBuildArgs& a, hipStream_t st, int old_nbodies);

// contact.hip
void launch_contact(const StepArgs* args, int grid, int precision, bool batched, bool periodic, int block,
                    hipStream_t st);

// integrate.hip
void launch_integrate(const StepArgs* args, int grid, int precision, bool batched, bool periodic, int block,
                      hipStream_t st);
void launch_body_forces(const StepArgs& a, int precision, double* f3, double* t3, hipStream_t st);


}  // namespace dem
