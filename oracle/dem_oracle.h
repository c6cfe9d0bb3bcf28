/*
 * dem_oracle.h -- plain single-threaded FP64 reference implementation of one
 * soft-sphere DEM timestep (spheres + axis-aligned walls, linear
 * Cundall-Strack law, damped leapfrog), written from the Yade DEM
 * documentation (3rd ed., arXiv 2301.00611).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU path.
 * It shares no source with it: only tests/, the smoke check and the CPU
 * baseline leg of the benchmark may load it.  The product path never calls it.
 *
 * Conventions (each one is a reading of the documentation; the full list is
 * in the repository's design notes):
 *   - one id space over walls and spheres, in insertion order from 0;
 *   - a sphere-sphere contact has #1 = lower id, #2 = higher id; a
 *     wall-sphere contact always has the wall as #1 (Ig2_Wall_Sphere_ScGeom);
 *   - the normal points from #1 to #2 (class reference: ScGeom.normal);
 *   - forces stored per contact are those sustained by #2
 *     (class reference: FrictPhys.normalForce / shearForce);
 *   - 3x3 matrices are row-major; the cell vectors are the COLUMNS of H
 *     (section 2.1.6, Cell.hSize).
 *
 * Every function returns ORC_OK (0) or an error code; orc_last_error() gives
 * a message.  Buffers are caller-owned; the scene deep-copies its inputs.
 */
#ifndef DEM_ORACLE_H
#define DEM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum {
    ORC_OK = 0,
    ORC_EINVAL = 1,     /* bad argument */
    ORC_ERANGE = 2,     /* id out of range */
    ORC_ECAPACITY = 4,  /* output buffer too small */
    ORC_ENOMEM = 5,
    ORC_ENONFINITE = 7, /* NaN/Inf in the state after a step */
    ORC_EPERIODIC = 8   /* a pair touches through more than one periodic image */
};

typedef struct orc_scene orc_scene;

typedef struct {
    double dt;           /* timestep [s] */
    double gravity[3];   /* NewtonIntegrator.gravity [m/s^2] */
    double damping;      /* Cundall non-viscous damping coefficient (eq. 2.9) */
    int damp_rot;        /* 1: apply eq. 2.9 to torques as well */
    int periodic;        /* 1: periodic cell (section 2.1.6) */
    double hsize[9];     /* H, columns are the cell vectors */
    double velgrad[9];   /* velocity gradient L */
    int homo_deform;     /* Cell.homoDeform: 0, 1 or 2 */
} orc_params;

typedef struct {
    long id1, id2;       /* #1, #2 (wall is #1 for wall-sphere) */
    int cell[3];         /* periodic image of #2 (Interaction.cellDist) */
    int is_wall;         /* 1 for a wall-sphere contact */
    double normal[3];    /* from #1 to #2 */
    double pen;          /* overlap, > 0 */
    double point[3];     /* contact point */
    double fn[3];        /* normal force on #2 */
    double fs[3];        /* shear force on #2 (after the Coulomb cap) */
    double kn, ks;
} orc_contact;

orc_scene* orc_create(const orc_params* p);
void orc_destroy(orc_scene* s);

/* FrictMat: density [kg/m3], young [Pa], poisson [-], frictionAngle [rad]. */
int orc_add_material(orc_scene* s, double density, double young, double poisson,
                     double friction_angle, int* out_mat);
/* ViscElMat given by contact time tc [s], normal and tangential restitution
 * coefficients en, et in (0, 1], frictionAngle [rad] (Law2_ScGeom_ViscElPhys_Basic,
 * Ip2_ViscElMat_ViscElMat_ViscElPhys); young and poisson take the class's
 * defaults (1e9, 0.25), used only by the P-wave step.  A scene's bodies must
 * all use materials of one kind (orc_step fails with ORC_EINVAL otherwise). */
int orc_add_viscel_material(orc_scene* s, double density, double tc, double en, double et,
                            double friction_angle, int* out_mat);
/* n spheres; vel3 / angvel3 / mat / blocked may be NULL.  blocked bits:
 * 1,2,4 = x,y,z translation, 8,16,32 = x,y,z rotation (State.blockedDOFs). */
int orc_add_spheres(orc_scene* s, long n, const double* pos3, const double* radius,
                    const double* vel3, const double* angvel3, const int* mat,
                    int default_mat, const unsigned char* blocked, long* out_first_id);
/* infinite plane normal to `axis` at coordinate `position`; sense -1/0/+1. */
int orc_add_wall(orc_scene* s, int axis, double position, int sense, int mat, long* out_id);

/* Fixed boundaries besides planes: an axis-aligned box (Box, centre and
 * half-sizes, Ig2_Box_Sphere_ScGeom) and a triangle (Facet, vertices v0, v1,
 * v2, two-sided, Ig2_Facet_Sphere_ScGeom with reference radius 2r).  Like a
 * wall, a boundary is #1 of its contacts. */
int orc_add_box(orc_scene* s, const double* center3, const double* half3, int mat, long* out_id);
int orc_add_facet(orc_scene* s, const double* v0, const double* v1, const double* v2, int mat, long* out_id);
/* utils.PWaveTimeStep: min over spheres of r*sqrt(rho/E). */
int orc_pwave_dt(const orc_scene* s, double* out);
int orc_step(orc_scene* s, long nsteps);

long orc_num_bodies(const orc_scene* s);
long orc_num_contacts(const orc_scene* s);
int orc_get_counters(const orc_scene* s, long* iter, double* time);

/* All bodies in id order; any pointer may be NULL.  Forces/torques are the
 * resultants of the last step's contacts (gravity not included).  For a wall,
 * pos3[axis] holds its position and the rest is 0; a box reports its centre
 * and a facet its centroid. */
int orc_get_state(const orc_scene* s, double* pos3, double* vel3, double* angvel3,
                  double* ori4, double* force3, double* torque3);
/* Mass and scalar inertia of every body (0 for walls). */
int orc_get_mass(const orc_scene* s, double* mass, double* inertia);
/* Overwrite sphere state (walls are skipped); any pointer may be NULL. */
int orc_set_state(orc_scene* s, const double* pos3, const double* vel3,
                  const double* angvel3, const double* ori4);

/* Real contacts of the last step, sorted by (min id, max id, cell). */
int orc_get_contacts(const orc_scene* s, long capacity, orc_contact* out, long* out_count);
/* Replace the shear history: n records (id1,id2,cell,Fs,n_prev).  Used by
 * tests to start two implementations from the same history. */
int orc_set_contacts(orc_scene* s, long n, const long* id1, const long* id2,
                     const int* cell3, const double* fs3, const double* nprev3);

/* kinetic, kin_rot, elastic, grav_work, damp_dissip, plastic_dissip, total,
 * visc_dissip (cumulative dashpot work of the visco-elastic law; in total) */
int orc_get_energy(const orc_scene* s, double* out8);
int orc_get_cell(const orc_scene* s, double* hsize9, double* trsf9);
/* Love-Weber stress of the last step's sphere-sphere contacts (force on #2
 * times the branch vector from #2 to #1, over V; V <= 0 takes the periodic
 * cell's volume). */
int orc_get_stress(const orc_scene* s, double volume, double* sigma9);

/* O.dt and Cell.velGrad, changed between steps. */
int orc_set_dt(orc_scene* s, double dt);
int orc_set_velgrad(orc_scene* s, const double* velgrad9);
/* Real pairs at the CURRENT positions (no step), by brute force. */
int orc_detect_pairs(const orc_scene* s, long capacity, long* id1, long* id2,
                     int* cell3, long* out_count);

/* Spot mode for large scenes: for k sphere ids, evaluate their contacts
 * against all bodies (O(k*N)) from the current state and shear history, and
 * return what one step would give for those bodies: resultant force/torque
 * and the integrated state.  Nothing in the scene changes.  n_contacts gets
 * the number of real contacts of each sampled body, fmag_sum the sum of
 * their force magnitudes (the scale of a near-cancelling resultant). */
int orc_spot_step(const orc_scene* s, long k, const long* ids, double* force3,
                  double* torque3, double* pos3, double* vel3, double* angvel3,
                  double* ori4, long* n_contacts, double* fmag_sum);

const char* orc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
