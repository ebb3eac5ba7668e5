/*
 * elbm_oracle.h -- plain FP64 CPU oracle for grid-refined KBC lattice Boltzmann
 * (Dorschner, Frapolli, Chikatamarla, Karlin, "Grid refinement for entropic
 * lattice Boltzmann models", arXiv:1608.06915).
 *
 * TEST INFRASTRUCTURE.  This library is the independent reference against which
 * the HIP path is checked.  Only the test suite, the smoke check and the CPU leg
 * of the benchmark may load it.  It shares no code, headers, tables or constants
 * with the HIP library.
 *
 * Conventions (also the public conventions of the HIP library, written there
 * independently):
 *   - Velocity index: i = (cx+1) + 3(cy+1) [+ 9(cz+1)], Q = 9 (D=2) or 27 (D=3);
 *     the opposite velocity of i is Q-1-i.
 *   - Level l node coordinates are integers in units of the level-l spacing
 *     (coarse spacing / 2^l).  A periodic axis with N coarse nodes has period
 *     N*2^l at level l; a non-periodic axis has nodes 0 .. (N-1)*2^l.
 *   - Dense per-level arrays cover the level's index box (ora_level_box),
 *     x fastest; vector fields are [component][box].
 *   - Face numbering: 0:-x 1:+x 2:-y 3:+y 4:-z 5:+z.
 */
#ifndef ELBM_ORACLE_H
#define ELBM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ora ora_t;

enum { ORA_FACE_PERIODIC = 0, ORA_FACE_WALL = 1, ORA_FACE_INLET = 2, ORA_FACE_OUTFLOW = 3 };

ora_t *ora_create(int D, const int64_t N[3], const int periodic[3], double nu0, int n_levels);
void ora_destroy(ora_t *o);
const char *ora_error(const ora_t *o);
int ora_set_face(ora_t *o, int face, int kind, const double u[3]);
int ora_add_box(ora_t *o, int level, const int64_t lo[3], const int64_t hi[3]);
int ora_set_solid(ora_t *o, int level, const int64_t lo[3], const int64_t n[3], const uint8_t *mask);
int ora_set_force_uniform(ora_t *o, const double F[3]);
int ora_finalize(ora_t *o);
int ora_level_box(const ora_t *o, int level, int64_t lo[3], int64_t n[3]);
int ora_level_info(const ora_t *o, int level, int64_t *n_nodes, int64_t *n_fluid, double *beta);
int ora_node_class(const ora_t *o, int level, int32_t *out);
int ora_weights(const ora_t *o, int level, double *out);
int ora_init(ora_t *o, int level, const double *rho, const double *u, const double *noise);
int ora_set_force_field(ora_t *o, int level, const double *F);
int ora_set_f(ora_t *o, int level, const double *f);
int ora_advance(ora_t *o, int n_coarse_steps);
int ora_get_f(const ora_t *o, int level, double *out);
int ora_moments(const ora_t *o, int level, double *rho, double *u, double *gamma);
int ora_sample_f(const ora_t *o, int level, int64_t n, const int64_t *coords, double *out);
int ora_reduce(const ora_t *o, double *mass, double mom[3]);
int ora_drag(ora_t *o, int level, double F[3], int64_t *steps, int reset);
/* Sec. III.C steps 3-4 on given post-stream states of levels lp, lp+1 (dense [Q][box],
 * in/out; non-finite = missing population) */
int ora_couple_states(ora_t *o, int lp, double *gp, double *gc);
/* Re-meshing: carry the state of src (same domain, levels, parameters, boundaries;
 * other refinement blocks) over to dst at a coarse-step boundary */
int ora_transfer_state(ora_t *dst, const ora_t *src);

/* node-level primitives */
void ora_feq(int D, double rho, const double u[3], double *feq);
double ora_kbc(int D, double beta, const double *f, const double F[3], double *out, double *ds,
               double *dh);
double ora_beta(double nu);
/* threads the node loops run on (1 unless built with OpenMP) */
int ora_threads(void);

/* discrete adjoint (reverse mode of the coarse step above) */
void ora_kbc_adj(int D, double beta, const double *f, const double F[3], const double *lo, double *lf,
                 double lF[3]);
int ora_adjoint_run(ora_t *o, int n_coarse_steps, int objective, int body_level, const double dir[3],
                    double *J_out);
int ora_adjoint_state(const ora_t *o, int level, double *out);
int ora_adjoint_force(const ora_t *o, int level, double *out);
int ora_init_adjoint_u(int D, int64_t n, const double *rho, const double *u, const double *noise,
                       const double *lam, double *out);

#ifdef __cplusplus
}
#endif
#endif
