/*
 * dem.h -- C ABI of libdem_hip.so, an MI355X (gfx950) implementation of one
 * soft-sphere discrete-element timestep over spheres and axis-aligned walls,
 * as described in the Yade DEM documentation (3rd ed., arXiv 2301.00611):
 *
 *   collider (section 2.1.1, InsertionSortCollider role)  -> Morton sort +
 *       cell-list sweep on the GPU, re-run only when a body may have moved
 *       farther than the Verlet distance (eq. 2.3-2.4);
 *   Ig2_Sphere_Sphere_ScGeom / Ig2_Wall_Sphere_ScGeom (section 2.1.3, class
 *       ScGeom): normal, overlap, contact point, shear update;
 *   Ip2_FrictMat_FrictMat_FrictPhys (section 2.1.2): kn, ks, tan(phi);
 *   Law2_ScGeom_FrictPhys_CundallStrack (section 2.1.4): linear normal force,
 *       incremental shear spring, Mohr-Coulomb cap;
 *   force/torque sum (ForceContainer), deterministic, no float atomics;
 *   NewtonIntegrator (section 2.1.5): gravity, Cundall damping eq. 2.9,
 *       leapfrog, spherical rotation; periodic Cell (section 2.1.6).
 *
 * Conventions
 *   Ids: one id space over walls and spheres, in insertion order from 0
 *     (O.bodies.append returns sequential ids).  Ids never change; the
 *     library reorders bodies internally but always speaks ids.
 *   Contacts: sphere-sphere contacts have #1 = lower id; a wall-sphere
 *     contact always has the wall as #1.  The normal points from #1 to #2
 *     (class ScGeom.normal).  Forces are those sustained by #2 (class
 *     FrictPhys.normalForce / shearForce).  `cell` is the periodic image of
 *     #2 (Interaction.cellDist).
 *   Matrices are 3x3 row-major; the cell vectors are the columns of hsize.
 *   Units are SI.  All floating-point arguments are double.
 *
 * Ownership
 *   Every input array is deep-copied before the call returns.  Outputs go to
 *   caller-allocated buffers whose size the caller states; DEM_ECAPACITY
 *   reports the size needed.  The scene (or batch) owns all device memory;
 *   dem_destroy / dem_batch_destroy free it.  A batch's scene views own
 *   nothing and must not be destroyed.
 *
 * Errors
 *   Every call returns DEM_OK (0) or a dem_status code; dem_last_error()
 *   returns a thread-local message valid until the next call on that thread.
 *   After any error except DEM_EDEVICE the scene is unchanged and usable.
 *
 * Threading: a scene is not thread-safe; distinct scenes may be used from
 * distinct threads.
 */
#ifndef DEM_H
#define DEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DEM_ABI_VERSION 1

typedef int32_t dem_status;
enum {
    DEM_OK = 0,
    DEM_EINVAL = 1,       /* bad argument (NULL, n < 0, r <= 0, bad axis/sense, ...) */
    DEM_ERANGE = 2,       /* body id out of range */
    DEM_ENOENT = 3,       /* no such object */
    DEM_ECAPACITY = 4,    /* caller buffer too small; *out_count holds the size needed */
    DEM_ENOMEM = 5,       /* device or host allocation failed */
    DEM_EDEVICE = 6,      /* HIP runtime error; message holds the HIP error string */
    DEM_ENONFINITE = 7,   /* NaN/Inf in positions or velocities after a step */
    DEM_EPERIODIC = 8,    /* periodic cell too small for the spheres and Verlet distance */
    DEM_EUNSTABLE = 9,    /* overlap exceeded a sphere radius ("numerically exploding");
                             a centre inside a box is not counted */
    DEM_EBUSY = 10        /* an asynchronous step is in flight (dem_step_async) */
};

enum { DEM_FP64 = 0, DEM_FP32_MIXED = 1 };

typedef struct dem_scene dem_scene;
typedef struct dem_batch dem_batch;

typedef struct {
    double dt;            /* timestep [s] (> 0) */
    double gravity[3];    /* NewtonIntegrator.gravity [m/s^2] */
    double damping;       /* NewtonIntegrator.damping, Cundall lambda in [0, 1) */
    int32_t damp_rot;     /* 1: apply eq. 2.9 to torques too (default 1) */
    double verlet_dist;   /* Delta L [m]; < 0 means -verlet_dist * (smallest radius)
                             (InsertionSortCollider.verletDist, default -0.5) */
    int32_t precision;    /* DEM_FP64 or DEM_FP32_MIXED */
    int32_t periodic;     /* 1: periodic cell (no walls allowed) */
    double hsize[9];      /* Cell.hSize, columns are the cell vectors */
    double velgrad[9];    /* Cell.velGrad */
    int32_t homo_deform;  /* Cell.homoDeform 0, 1 or 2 (default 2) */
    int32_t track_energy; /* 1: accumulate the energy terms every step */
    int32_t device;       /* HIP device ordinal */
    void* stream;         /* hipStream_t to run on, or NULL for a library-owned stream */
} dem_params;

/* One real contact.  Under the visco-elastic law fn holds the spring and
 * the normal dashpot (k_n pen - c_n u_n) n, fs the spring's and the shear
 * dashpot's force, and kn, ks the pair's visco-elastic stiffnesses; the shear
 * history (dem_history) holds the spring's part only. */
typedef struct {
    int64_t id1, id2;
    int32_t cell[3];
    int32_t is_wall;
    double normal[3];     /* unit, from #1 to #2 */
    double pen;           /* overlap (> 0 for a touching pair) */
    double point[3];      /* contact point, middle of the overlap */
    double fn[3];         /* normal force on #2 */
    double fs[3];         /* shear force on #2 (after the Coulomb cap) */
    double kn, ks;
} dem_contact;

/* Shear history record, for checkpoint/restore and tests. */
typedef struct {
    int64_t id1, id2;
    int32_t cell[3];
    int32_t pad;
    double fs[3];         /* shear force on #2 */
    double nprev[3];      /* normal of the previous step */
} dem_history;

typedef struct {
    double kinetic;        /* sum 1/2 m |v-|^2 of the last step */
    double kin_rot;        /* sum 1/2 I |w-|^2 of the last step */
    double elastic;        /* sum 1/2 |Fn|^2/kn + 1/2 |Fs|^2/ks of the last step */
    double grav_work;      /* cumulative work of gravity, negated */
    double damp_dissip;    /* cumulative energy removed by eq. 2.9 */
    double plastic_dissip; /* cumulative Coulomb slip work */
    double total;          /* sum of the above and visc_dissip */
    double visc_dissip;    /* cumulative work of the visco-elastic law's dashpots */
} dem_energy;

typedef struct {
    int64_t iter;            /* steps done */
    double time;             /* simulated time [s] */
    int64_t n_spheres, n_walls;
    int64_t n_contacts_ss;   /* real sphere-sphere contacts at the last step */
    int64_t n_contacts_sw;   /* real sphere-wall contacts at the last step */
    int64_t n_candidates;    /* candidate pairs kept by the last broad phase */
    int64_t rebuilds;        /* broad-phase runs so far */
    int64_t contact_steps;   /* sum over steps of the real contacts */
    double coordination;     /* 2 C_ss / N_spheres (utils.avgNumInteractions) */
    double verlet_dist;      /* Delta L in use [m] */
    double max_overlap_ratio; /* largest overlap / smaller radius at the last step; past 1
                                 the run is exploding (class InsertionSortCollider,
                                 periodic limitations) and dem_step fails */
} dem_stats;

/* Performance knobs; none of them changes any result (positions,
 * velocities, forces and contacts are bit for bit the same whatever the
 * setting; only the per-block energy partial sums regroup). */
typedef struct {
    int32_t block_contact;   /* threads per block of the contact kernel: 64..1024, multiple of 64 */
    int32_t block_integrate; /* same for the integrate kernel */
    int32_t chunk;           /* steps per captured HIP graph: even, 2..4096 */
    int32_t pad;
    double verlet_factor;    /* Delta L = factor x smallest radius, every scene (0 = keep verlet_dist) */
    double ms_per_step;      /* wall time per step measured by the autotuner, 0 if never measured */
} dem_tuning;

int32_t dem_abi_version(void);
const char* dem_last_error(void);
/* Fill *p with the documentation's defaults (damping 0.2, verletDist -0.5,
 * homoDeform 2, FP64, energy tracking off, device 0, no stream, dt = 0). */
void dem_params_default(dem_params* p);

dem_status dem_create(const dem_params* p, dem_scene** out);
dem_status dem_destroy(dem_scene* s);

/* FrictMat (section 2.3.1 materials): density > 0 [kg/m3], young > 0 [Pa],
 * poisson in (-1, 0.5], friction_angle in [0, pi/2) [rad]. */
dem_status dem_add_material(dem_scene* s, double density, double young, double poisson,
                            double friction_angle, int32_t* out_mat);
/* ViscElMat (class ViscElMat; Ip2_ViscElMat_ViscElMat_ViscElPhys and
 * Law2_ScGeom_ViscElPhys_Basic): density > 0, contact time tc > 0 [s],
 * normal and tangential restitution coefficients en, et in (0, 1],
 * friction_angle as above.  A pair takes the means of the two materials'
 * tc, en, et and its reduced mass m (the sphere's own against a boundary):
 * kn = m (pi^2 + ln^2 en)/tc^2, cn = -2 m ln(en)/tc, ks = 2/7 m (pi^2 +
 * ln^2 et)/tc^2, cs = -2/7 m ln(et)/tc (the analytic two-sphere solution of
 * getViscoelasticFromSpheresInteraction).  young and poisson take the class
 * defaults 1e9 and 0.25, used only by dem_pwave_dt.  The bodies of one scene
 * must all use materials of one kind (dem_step fails with DEM_EINVAL
 * otherwise); the stiffness timestep, its timestepper and the controlled cell
 * are refused (DEM_EINVAL) while visco-elastic materials exist. */
dem_status dem_add_viscel_material(dem_scene* s, double density, double tc, double en, double et,
                                   double friction_angle, int32_t* out_mat);
/* Append n spheres (ids out_first_id .. +n-1).  pos3 [n*3], radius [n] are
 * required; vel3, angvel3 [n*3], mat [n], blocked [n] may be NULL (zero /
 * default_mat / none).  blocked bits 1,2,4 = x,y,z translation, 8,16,32 =
 * rotation (State.blockedDOFs): a blocked component keeps its velocity.
 * Mass = 4/3 pi r^3 rho, inertia = 2 m r^2 / 5.  Host buffers. */
dem_status dem_add_spheres(dem_scene* s, int64_t n, const double* pos3, const double* radius,
                           const double* vel3, const double* angvel3, const int32_t* mat,
                           int32_t default_mat, const uint8_t* blocked, int64_t* out_first_id);
/* Infinite plane normal to axis (0,1,2) at `position`; sense -1/0/+1
 * (class Wall): the side(s) it interacts with.  Walls do not move. */
dem_status dem_add_wall(dem_scene* s, int32_t axis, double position, int32_t sense, int32_t mat,
                        int64_t* out_id);
/* Fixed boundaries besides planes; like a wall each is #1 of its contacts,
 * takes an id in the same sequence and is not moved.
 *  - dem_add_box: an axis-aligned box (class Box, Ig2_Box_Sphere_ScGeom)
 *    with the given centre and half-sizes (> 0).  A sphere whose centre is
 *    outside touches it when closer than r to the box: normal from the
 *    closest point towards the centre, overlap r - distance; a centre inside
 *    the box is pushed out through the nearest face (overlap r + depth).
 *    Reference radius: the sphere's (a virtual sphere of the same radius).
 *  - dem_add_facet: a triangle v0, v1, v2 (class Facet,
 *    Ig2_Facet_Sphere_ScGeom), two-sided: normal from the closest point of
 *    the triangle towards the centre (the face normal (v1 - v0) x (v2 - v0)
 *    when the centre lies on it), overlap r - distance; reference radius
 *    twice the sphere's.  A degenerate triangle is DEM_EINVAL.
 * At most 64 boundaries (planes included) per scene; none in a periodic
 * cell.  dem_get_state reports a box's centre and a facet's centroid. */
dem_status dem_add_box(dem_scene* s, const double* center3, const double* half3, int32_t mat, int64_t* out_id);
dem_status dem_add_facet(dem_scene* s, const double* v0, const double* v1, const double* v2, int32_t mat,
                         int64_t* out_id);

/* utils.PWaveTimeStep: min over spheres of r / sqrt(E / rho). */
dem_status dem_pwave_dt(dem_scene* s, double* out);
dem_status dem_set_dt(dem_scene* s, double dt);
/* Periodic scenes: replace Cell.velGrad (applied from the next step). */
dem_status dem_set_velgrad(dem_scene* s, const double* velgrad9);
dem_status dem_get_cell(dem_scene* s, double* hsize9, double* trsf9);

/* Advance nsteps steps (O.run(n, wait=True)); returns when they are done.
 * nsteps = 0 advances nothing but runs a pending broad phase (after bodies
 * were added or moved, or when the last step asked for one), so that the
 * next step starts from an up-to-date candidate list. */
dem_status dem_step(dem_scene* s, int64_t nsteps);
/* O.run(n) without waiting (section 2.2.1 running simulations): the steps
 * run on a library thread; until dem_wait returns, every other call on this
 * scene (or its batch) returns DEM_EBUSY.  dem_wait (O.wait) joins and
 * returns the status (and message) the steps ended with; it returns DEM_OK
 * at once when nothing is in flight.  dem_destroy waits first. */
dem_status dem_step_async(dem_scene* s, int64_t nsteps);
dem_status dem_wait(dem_scene* s);

/* State of `count` bodies starting at id first_id, in id order, into HOST
 * buffers; any pointer may be NULL.  force3/torque3 are the resultants of
 * the last step's contacts (gravity excluded; walls get the reaction).  For
 * a wall, pos3[axis] is its position and the rest is 0. */
dem_status dem_get_state(dem_scene* s, int64_t first_id, int64_t count, double* pos3, double* vel3,
                         double* angvel3, double* ori4, double* force3, double* torque3);
/* Same, into DEVICE buffers on the scene's device (e.g. torch tensors); the
 * copy is ordered on the scene's stream and complete when the call returns. */
dem_status dem_get_state_device(dem_scene* s, int64_t first_id, int64_t count, double* pos3,
                                double* vel3, double* angvel3, double* ori4);
/* Overwrite the state of every sphere (ids in order; walls skipped); any
 * pointer may be NULL.  Forces a broad-phase run before the next step. */
dem_status dem_set_state(dem_scene* s, const double* pos3, const double* vel3,
                         const double* angvel3, const double* ori4);
/* Mass and inertia of every body (0 for walls). */
dem_status dem_get_mass(dem_scene* s, double* mass, double* inertia);

/* Real contacts of the last step, sorted by (min id, max id, cell). */
dem_status dem_get_contacts(dem_scene* s, int64_t capacity, dem_contact* out, int64_t* out_count);
/* O.interactions[id1, id2] (class InteractionContainer): the real contact
 * between two bodies, looked up symmetrically (id1, id2 in either order;
 * cell3 = image of id2 seen from id1, NULL = (0,0,0)).  DEM_ERANGE for an
 * id out of range, DEM_ENOENT when the pair is not in contact.  Reads the
 * contact list back from the device: meant for inspection, not for loops. */
dem_status dem_get_interaction(dem_scene* s, int64_t id1, int64_t id2, const int32_t* cell3,
                               dem_contact* out);
/* Shear history (all real contacts); dem_set_history replaces it and forces
 * a broad-phase run (the records are carried onto the new candidate list). */
dem_status dem_get_history(dem_scene* s, int64_t capacity, dem_history* out, int64_t* out_count);
dem_status dem_set_history(dem_scene* s, int64_t n, const dem_history* in);

dem_status dem_get_energy(dem_scene* s, dem_energy* out);
/* utils.getStress (Love-Weber): sigma_ij = (1/V) sum over the real
 * sphere-sphere contacts of the last step of f_i l_j, f the force on #2 and
 * l the branch vector from #2 to #1 (negative under compression).  Wall
 * contacts are left out.  volume <= 0 takes the periodic cell's volume
 * (DEM_EINVAL for an aperiodic scene).  sigma9 is a host buffer of 9
 * doubles, row-major. */
dem_status dem_get_stress(dem_scene* s, double volume, double* sigma9);
/* dem_get_stress for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * stress, from the same contacts, with its partial sums in a fixed device
 * array of the library (1025 x 9 doubles, 73,800 bytes, one per GPU, kept
 * until the process ends) instead of a buffer sized to the scene; it calls
 * no hipMalloc or hipFree and no allocating routine.  The sums are taken in
 * another fixed order than dem_get_stress's, so the two agree to rounding
 * (relative 1e-12), not bit for bit; each is deterministic.  Limits: at most
 * 67,108,864 candidate pairs (DEM_EINVAL beyond); the device state must be
 * current (DEM_EINVAL when bodies were added or the state set since the last
 * step, which dem_get_stress would upload).  Calls that overlap on one GPU
 * (other threads, other scenes) share the array and race. */
dem_status dem_get_stress_noalloc(dem_scene* s, double volume, double* sigma9);
dem_status dem_get_stats(dem_scene* s, dem_stats* out);

/* utils.unbalancedForce (section 5 utility reference): the mean (use_max =
 * 0) or largest (use_max = 1) magnitude of the resultant contact force over
 * the dynamic spheres (not all six DOFs blocked; gravity is not part of
 * it), divided by the mean |F_n + F_s| over the last step's real contacts
 * (walls included).  *out is NaN when either set is empty.  Computed on the
 * device with fixed-order sums. */
dem_status dem_get_unbalanced_force(dem_scene* s, int32_t use_max, double* out);
/* GlobalStiffnessTimeStepper (eqs. 2.12-2.14): safety x the smallest
 * sqrt(2) sqrt(m / K_ii) over the dynamic spheres' unblocked DOFs, with the
 * translational stiffness K_ii = sum over the body's contacts of
 * (k_n - k_s) n_i^2 + k_s and the rotational one sum k_s r^2 (1 - n_i^2)
 * against the inertia, from the last step's contacts; safety x the P-wave
 * timestep when there is no contact.  safety in (0, 1]. */
dem_status dem_stiffness_dt(dem_scene* s, double safety, double* out);
/* Let the stiffness timestepper set dt before every step whose iteration
 * count is a multiple of `interval` (timeStepUpdateInterval); interval 0
 * turns it off.  Not available on batch views. */
dem_status dem_set_stiffness_timestepper(dem_scene* s, double safety, int64_t interval);

/* Stress/strain-controlled periodic cell (PeriTriaxController driven by the
 * packing stiffness).  After every step that makes the iteration count a
 * multiple of glob_update, the cell is steered from the last step's
 * contacts: with the Love-Weber stress sigma, the normal springs' modulus
 * M_i = (1/V) sum over sphere-sphere contacts of k_n (d_i n_i)^2 (d the
 * centre distance vector) and T = glob_update dt, a stress axis (bit i of
 * stress_mask set) gets the strain rate (1 - grow_damping)(goal_i -
 * sigma_ii) / (M_i T) (the full rate towards the goal's sign while
 * M_i = 0), a strain axis (strain = log of the cell transformation's
 * diagonal, relative to the initial cell) the rate (goal_i - strain_i) / T;
 * rates are capped at max_strain_rate and the velocity gradient becomes
 * diag(rates).  The goal is reached when every stress axis is within
 * max(abs_stress_tol, rel_stress_tol |goal_i|), every strain axis within
 * 1e-6 and the unbalanced force is at most max_unbalanced; the cell then
 * stops (zero velocity gradient) and, with stop_when_done, dem_step returns
 * early (dem_get_stats gives the steps done).  Periodic scenes only. */
typedef struct {
    double goal[3];            /* stress [Pa] or strain [-] per axis */
    int32_t stress_mask;       /* bit i: axis i is stress-controlled */
    int32_t glob_update;       /* steps between updates, >= 1 (default 5) */
    double max_strain_rate[3]; /* [1/s], > 0 (default 1) */
    double grow_damping;       /* in [0, 1) (default 0.25) */
    double max_unbalanced;     /* default 1e-4 */
    double abs_stress_tol;     /* [Pa], default 1e3 */
    double rel_stress_tol;     /* default 3e-5 */
    int32_t stop_when_done;
    int32_t pad;
} dem_peri_triax;
typedef struct {
    double stress[3];          /* diagonal of the stress at the last update [Pa] */
    double strain[3];          /* log of the transformation's diagonal */
    double strain_rate[3];     /* the velocity gradient's diagonal now in use [1/s] */
    double stiff[3];           /* M_i at the last update [Pa] */
    double unbalanced;         /* at the last update */
    int64_t updates;
    int32_t done;              /* the goal was reached at the last update */
    int32_t active;
} dem_peri_triax_state;

/* PeriIsoCompressor with keepProportions (class PeriIsoCompressor: stresses,
 * globalUpdateInt, maxUnbalanced, state, sigma, currUnbalanced): the cell is
 * compressed or dilated isotropically until the mean stress tr(sigma)/3
 * reaches stresses[0], then stresses[1], ... .  The law is the controlled
 * cell's (dem_set_peri_triax) applied to the mean: every global_update-th
 * step one strain rate (1 - grow_damping)(goal - sigma_m)/(M_m T) for all
 * three axes, M_m the mean of the normal springs' modulus per axis, T =
 * global_update dt, +-max_strain_rate while M_m = 0, capped at
 * max_strain_rate.  A stress is reached when |goal - sigma_m| <=
 * max(abs_stress_tol, rel_stress_tol |goal|) and the unbalanced force is at
 * most max_unbalanced; the next stress is then driven to from the same
 * update; after the last one the cell stops, and with stop_when_done
 * dem_step returns there (the doneHook's usual pause).  It replaces the
 * controlled cell of dem_set_peri_triax (one controller per scene). */
#define DEM_MAX_STRESS_SERIES 8
typedef struct {
    int32_t n_stresses;           /* 1 .. DEM_MAX_STRESS_SERIES */
    int32_t global_update;        /* globalUpdateInt, >= 1 (default 20) */
    double stresses[DEM_MAX_STRESS_SERIES]; /* [Pa], negative in compression */
    double max_strain_rate;       /* > 0 [1/s] (default 1) */
    double grow_damping;          /* [0, 1) (default 0.25) */
    double max_unbalanced;        /* maxUnbalanced (default 1e-4) */
    double abs_stress_tol;        /* [Pa] (default 1e3) */
    double rel_stress_tol;        /* (default 3e-5) */
    int32_t stop_when_done;
    int32_t pad_;
} dem_peri_iso;                   /* 136 bytes */

typedef struct {
    int32_t state;                /* index of the stress being driven to */
    int32_t done;                 /* 1 once the last stress is reached */
    double sigma;                 /* mean stress at the last update [Pa] */
    double stiff;                 /* mean normal-spring modulus at the last update [Pa] */
    double strain_rate;           /* the rate set on each axis [1/s] */
    double unbalanced;            /* currUnbalanced (NaN before the first update) */
    int64_t updates;
    int32_t active;               /* 1 while this compressor is the scene's controller */
    int32_t pad_;
} dem_peri_iso_state;             /* 56 bytes */

void dem_peri_triax_default(dem_peri_triax* c);
/* c = NULL switches the controller off (the velocity gradient stays). */
dem_status dem_set_peri_triax(dem_scene* s, const dem_peri_triax* c);
dem_status dem_get_peri_triax(dem_scene* s, dem_peri_triax_state* out);
/* The isotropic compressor; NULL switches the scene's controller off.  Same
 * scene requirements and refusals as dem_set_peri_triax; DEM_EINVAL for an
 * empty or too long series or a non-finite stress. */
void dem_peri_iso_default(dem_peri_iso* c);
dem_status dem_set_peri_iso(dem_scene* s, const dem_peri_iso* c);
dem_status dem_get_peri_iso(dem_scene* s, dem_peri_iso_state* out);

/* Average device duration [ms] of each kernel family over the last
 * dem_step call (names: "contact", "integrate", "rebuild"), measured with
 * HIP events when timing is on. */
dem_status dem_set_timing(dem_scene* s, int32_t on);
dem_status dem_get_timing(dem_scene* s, const char* name, double* avg_ms, int64_t* launches);

/* The autotuner (for the batched form above all, where scene sizes vary):
 * dem_autotune looks the workload up in the text cache file `cache_path`
 * (key: GPU architecture, precision, batched/periodic, log2 of the sphere
 * and candidate counts, number of scenes) and applies the stored setting;
 * without an entry it times `probe_steps` ordinary steps per candidate
 * setting, trying Verlet factors 0.05/0.1/0.25/0.5/1, block sizes
 * 128..1024 and chunks 16/32/64 one knob at a time, keeps the fastest and
 * appends it to the cache (NULL or "" = no cache).  A setting is charged its
 * broad phase at its rate: the window's time without its broad-phase runs,
 * plus the last run's cost over the steps between runs, estimated from the
 * growth of the largest Verlet account.  The probe steps advance the
 * simulation like any other steps.  dem_set_tuning on a batch view is
 * refused: use the batch calls. */
dem_status dem_get_tuning(dem_scene* s, dem_tuning* out);
dem_status dem_set_tuning(dem_scene* s, const dem_tuning* t);
dem_status dem_autotune(dem_scene* s, int64_t probe_steps, const char* cache_path, dem_tuning* out);

/* Batched scenes: n_scenes independent scenes advanced together by the same
 * kernels (one bodies arena, per-scene parameters).  per_scene[i].periodic
 * must be 0; precision, device and stream are taken from per_scene[0]. */
dem_status dem_batch_create(int32_t n_scenes, const dem_params* per_scene, dem_batch** out);
/* Non-owning view of scene i: use it with dem_add_*, dem_get_*, dem_pwave_dt.
 * dem_step on a view is refused: step the whole batch. */
dem_status dem_batch_scene(dem_batch* b, int32_t i, dem_scene** view);
dem_status dem_batch_step(dem_batch* b, int64_t nsteps);
dem_status dem_batch_stats(dem_batch* b, dem_stats* out);
dem_status dem_batch_set_tuning(dem_batch* b, const dem_tuning* t);
dem_status dem_batch_autotune(dem_batch* b, int64_t probe_steps, const char* cache_path, dem_tuning* out);
dem_status dem_batch_destroy(dem_batch* b);

#ifdef __cplusplus
}
#endif
#endif
