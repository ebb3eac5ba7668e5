/*
 * elbm_oracle.c -- plain FP64 CPU oracle for grid-refined KBC lattice Boltzmann.
 *
 * TEST INFRASTRUCTURE ONLY: the reference that the HIP library is checked against.
 * Only tests, the smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no code with the HIP path.
 *
 * Structure is chosen for checkability, not speed:
 *   - array-of-structs populations f[node][Q], double precision throughout;
 *   - explicit post-stream arrays g[node][Q] with one validity bit per population,
 *     so that "information is missing" (Sec. III.C, steps 1-2) is tracked
 *     mechanically and every use of a missing value is an error;
 *   - the refinement algorithm of Sec. III.C run as a literal recursion over levels;
 *   - node lists per level with a dense coordinate -> node map.
 *
 * Paper sections cited: Sec. II (LBE, Eq. f_equations; equilibrium Eq. feq_iso;
 * viscosity Eq. visc; moments Eq. moments; k/s/h split Eq. popSplit; mirror state
 * Eq. f_mirr; stabiliser Eq. gamma_min_approx), Sec. III.A (convective scaling,
 * relaxation rescaling, exact-difference forcing, non-equilibrium rescaling
 * Eq. f_neq_rescaling_iso), Sec. III.B (four-point interpolation Eq. interp),
 * Sec. III.C (five-step algorithm).
 *
 * Readings where the paper is silent (each listed in the design notes):
 *   R1 s-part = deviatoric second-order moments only, the trace goes to h.
 *   R2 D2Q9 KBC = the two-dimensional analogue of the D3Q27 model.
 *   R3 gamma := 2 when <dh|dh> = 0 or the ratio is not finite.
 *   R4 interpolation spacing dx = fine spacing, so the four points are coarse-aligned.
 *   R5 interface geometry: child box edges on parent nodes, outer/inner child layers
 *      at fine Chebyshev distance 0/1 from the child region boundary, parent ring at
 *      fine distance 2, no parent nodes deeper inside.
 *   R6 rescaling acts on post-stream, pre-collision states.
 *   R7 composite stencil: child bulk values where the child has bulk nodes, parent
 *      values (brought to child scale) elsewhere.
 *   R8 reported velocity with forcing = j/rho + du/2.
 *   R9 walls = halfway bounce-back, inlet = equilibrium at (1,U) for incoming
 *      populations, outflow = zero-gradient copy of incoming populations.
 *   R10 drag = momentum exchange on solid links, 2 c_i f'_i per link per step.
 *   R11 mass/momentum weights = owned volume with the cut half-way across the
 *      overlap (inner child layer counts by the fraction of its sub-cells that face
 *      child bulk nodes).
 */
#include "elbm_oracle.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OMAXL 8
#define OMAXQ 27
#define EXT_MARGIN 4

typedef struct {
  int64_t lo[3], hi[3];
} obox;

typedef struct {
  int64_t lo[3], n[3];
  uint8_t *mask;
} osolid;

typedef struct {
  /* user description */
  int nbox;
  obox *box;
  int nsol;
  osolid *sol;
  /* index box */
  int64_t blo[3], bn[3];
  /* distance grid (extended index box) */
  int64_t elo[3], en[3];
  int efull[3];
  uint8_t *dist; /* 255 = outside region or out of domain, else 0..3 */
  /* nodes */
  int32_t *id; /* dense over index box, -1 = absent */
  int64_t nn;
  int64_t *pos; /* [nn*3] */
  uint8_t *solid, *pd, *ring;
  double *w;
  /* state */
  double *f, *g, *gam, *force;
  uint8_t *vf, *vg;
  double beta;
  double drag[3];
  int64_t drag_steps;
  /* adjoint: of post-collision f, of post-stream g, of the per-node force */
  double *lf, *lg, *lF;
} olevel;

/* one recorded operation of a coarse step, with the inputs its reverse needs */
typedef struct {
  int op; /* 0 stream, 1 collide, 2 couple */
  int level, skip;
  double *g0, *g1;
} otape;

struct ora {
  int D, Q, L;
  int64_t N[3];
  int periodic[3];
  int face_kind[6];
  double face_u[6][3];
  double nu0;
  double Fu[3];
  int finalized;
  olevel lev[OMAXL];
  char err[512];
  /* velocity table */
  int c[OMAXQ][3];
  double W[OMAXQ];
  /* adjoint tape of the coarse step being recorded */
  int taping;
  otape *tape;
  int ntape, captape;
};

static int fail(ora_t *o, int code, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
#pragma omp critical(ora_fail)
  vsnprintf(o->err, sizeof(o->err), fmt, ap);
  va_end(ap);
  return code;
}

/* ---------------------------------------------------------------------------
 * Lattice: velocities c_i in {-1,0,1}^D, weights W_i = prod_a W_{c_ia} with
 * W_0 = 2/3, W_{+-1} = 1/6 (Sec. II.A, after Eq. feq_iso).  D2Q9 uses the same
 * product rule in two dimensions (reading R2).
 * ------------------------------------------------------------------------- */
static void lattice(int D, int c[OMAXQ][3], double W[OMAXQ]) {
  int Q = D == 2 ? 9 : 27;
  for (int i = 0; i < Q; ++i) {
    c[i][0] = i % 3 - 1;
    c[i][1] = (i / 3) % 3 - 1;
    c[i][2] = D == 3 ? i / 9 - 1 : 0;
    double w = 1.0;
    for (int a = 0; a < D; ++a) w *= (c[i][a] == 0) ? 2.0 / 3.0 : 1.0 / 6.0;
    W[i] = w;
  }
}

/* Eq. visc with c_s^2 = 1/3:  nu = (1/3)(1/(2 beta) - 1/2)  =>  beta = 1/(6 nu + 1). */
double ora_beta(double nu) { return 1.0 / (6.0 * nu + 1.0); }

/* threads the node loops use: 1 unless built with OpenMP */
int ora_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Eq. feq_iso: f_i^eq = rho W_i prod_a (2 - sqrt(1+3u_a^2)) ((2u_a + sqrt(1+3u_a^2))/(1-u_a))^{c_ia}. */
void ora_feq(int D, double rho, const double u[3], double *feq) {
  int c[OMAXQ][3];
  double W[OMAXQ];
  lattice(D, c, W);
  int Q = D == 2 ? 9 : 27;
  for (int i = 0; i < Q; ++i) {
    double v = rho * W[i];
    for (int a = 0; a < D; ++a) {
      double sq = sqrt(1.0 + 3.0 * u[a] * u[a]);
      double X = (2.0 * u[a] + sq) / (1.0 - u[a]);
      double p = (c[i][a] == 1) ? X : (c[i][a] == -1 ? 1.0 / X : 1.0);
      v *= (2.0 - sq) * p;
    }
    feq[i] = v;
  }
}

/* Shear part of a deviation d (reading R1): the population whose natural moments
 * (Eq. moments) vanish except the deviatoric second-order ones, which equal those
 * of d.  Closed forms (derived from Eq. moments and Eq. popSplit):
 *   D=2: N = sum d (cx^2 - cy^2), Pxy = sum d cx cy;
 *        (+-1,0): N/4, (0,+-1): -N/4, (s,t): s t Pxy/4, rest 0.
 *   D=3: Nxz = sum d (cx^2-cz^2), Nyz = sum d (cy^2-cz^2), Pxy, Pxz, Pyz;
 *        x-faces (2Nxz-Nyz)/6, y-faces (-Nxz+2Nyz)/6, z-faces (-Nxz-Nyz)/6,
 *        edge in the ab plane: c_a c_b P_ab/4, rest and corners 0. */
static void shear_part(int D, const int c[OMAXQ][3], const double *d, double *ds) {
  int Q = D == 2 ? 9 : 27;
  if (D == 2) {
    double N = 0, P = 0;
    for (int i = 0; i < Q; ++i) {
      N += d[i] * (c[i][0] * c[i][0] - c[i][1] * c[i][1]);
      P += d[i] * c[i][0] * c[i][1];
    }
    for (int i = 0; i < Q; ++i) {
      int ax = abs(c[i][0]), ay = abs(c[i][1]);
      if (ax + ay == 1) ds[i] = ax ? N / 4.0 : -N / 4.0;
      else if (ax + ay == 2) ds[i] = c[i][0] * c[i][1] * P / 4.0;
      else ds[i] = 0.0;
    }
    return;
  }
  double Nxz = 0, Nyz = 0, Pxy = 0, Pxz = 0, Pyz = 0;
  for (int i = 0; i < Q; ++i) {
    int x = c[i][0], y = c[i][1], z = c[i][2];
    Nxz += d[i] * (x * x - z * z);
    Nyz += d[i] * (y * y - z * z);
    Pxy += d[i] * x * y;
    Pxz += d[i] * x * z;
    Pyz += d[i] * y * z;
  }
  for (int i = 0; i < Q; ++i) {
    int x = c[i][0], y = c[i][1], z = c[i][2];
    int n = abs(x) + abs(y) + abs(z);
    double v = 0.0;
    if (n == 1) {
      if (x) v = (2.0 * Nxz - Nyz) / 6.0;
      else if (y) v = (-Nxz + 2.0 * Nyz) / 6.0;
      else v = (-Nxz - Nyz) / 6.0;
    } else if (n == 2) {
      if (!z) v = x * y * Pxy / 4.0;
      else if (!y) v = x * z * Pxz / 4.0;
      else v = y * z * Pyz / 4.0;
    }
    ds[i] = v;
  }
}

/* KBC collision with forcing at one node.
 *   Eq. f_equations + Eq. f_mirr give f' = f - beta (2 ds + gamma dh) (derived:
 *   f_mirr - f = -2 ds - gamma dh because k = k^eq).
 *   Eq. gamma_min_approx: gamma = 1/beta - (2 - 1/beta) <ds|dh>/<dh|dh>,
 *   <X|Y> = sum X_i Y_i / f_i^eq; reading R3 for <dh|dh> = 0.
 *   Exact-difference forcing (Sec. III.A): f' += f^eq(rho, u + du) - f^eq(rho, u),
 *   du = F / rho.
 * Returns gamma; ds, dh may be NULL. */
double ora_kbc(int D, double beta, const double *f, const double F[3], double *out, double *ds_out,
               double *dh_out) {
  int c[OMAXQ][3];
  double W[OMAXQ];
  lattice(D, c, W);
  int Q = D == 2 ? 9 : 27;
  double rho = 0, j[3] = {0, 0, 0};
  for (int i = 0; i < Q; ++i) {
    rho += f[i];
    for (int a = 0; a < 3; ++a) j[a] += c[i][a] * f[i];
  }
  double u[3] = {j[0] / rho, j[1] / rho, j[2] / rho};
  double feq[OMAXQ], d[OMAXQ], ds[OMAXQ], dh[OMAXQ];
  ora_feq(D, rho, u, feq);
  for (int i = 0; i < Q; ++i) d[i] = f[i] - feq[i];
  shear_part(D, c, d, ds);
  for (int i = 0; i < Q; ++i) dh[i] = d[i] - ds[i];
  double A = 0, B = 0;
  for (int i = 0; i < Q; ++i) {
    A += ds[i] * dh[i] / feq[i];
    B += dh[i] * dh[i] / feq[i];
  }
  double gamma = 2.0;
  if (B > 0.0) {
    gamma = 1.0 / beta - (2.0 - 1.0 / beta) * A / B;
    if (!isfinite(gamma)) gamma = 2.0;
  }
  for (int i = 0; i < Q; ++i) out[i] = f[i] - beta * (2.0 * ds[i] + gamma * dh[i]);
  if (F && (F[0] != 0.0 || F[1] != 0.0 || F[2] != 0.0)) {
    double u2[3] = {u[0] + F[0] / rho, u[1] + F[1] / rho, u[2] + F[2] / rho};
    double feq2[OMAXQ];
    ora_feq(D, rho, u2, feq2);
    for (int i = 0; i < Q; ++i) out[i] += feq2[i] - feq[i];
  }
  if (ds_out) memcpy(ds_out, ds, sizeof(double) * Q);
  if (dh_out) memcpy(dh_out, dh, sizeof(double) * Q);
  return gamma;
}

/* ---------------------------------------------------------------------------
 * Geometry
 * ------------------------------------------------------------------------- */
static int64_t lv_period(const ora_t *o, int l, int a) { return o->N[a] << l; }
static int64_t lv_extent(const ora_t *o, int l, int a) {
  if (a >= o->D) return 1;
  return o->periodic[a] ? (o->N[a] << l) : ((o->N[a] - 1) << l) + 1;
}
static int64_t wrapi(int64_t x, int64_t P) {
  int64_t r = x % P;
  return r < 0 ? r + P : r;
}
/* wrap periodic axes; returns 0 if out of domain on a non-periodic axis */
static int canon(const ora_t *o, int l, int64_t x[3]) {
  for (int a = 0; a < 3; ++a) {
    if (a >= o->D) {
      if (x[a] != 0) return 0;
      continue;
    }
    if (o->periodic[a]) x[a] = wrapi(x[a], lv_period(o, l, a));
    else if (x[a] < 0 || x[a] >= lv_extent(o, l, a)) return 0;
  }
  return 1;
}
static int box_full(const ora_t *o, int l, const obox *b, int a) {
  return o->periodic[a] && (b->hi[a] - b->lo[a] >= lv_period(o, l, a) - 1);
}
/* membership of a canonical in-domain position in the closed region of level l */
static int in_region(const ora_t *o, int l, const int64_t x[3]) {
  if (l == 0) return 1;
  const olevel *L = &o->lev[l];
  for (int b = 0; b < L->nbox; ++b) {
    const obox *bx = &L->box[b];
    int in = 1;
    for (int a = 0; a < o->D && in; ++a) {
      if (o->periodic[a]) {
        if (box_full(o, l, bx, a)) continue;
        int64_t off = wrapi(x[a] - bx->lo[a], lv_period(o, l, a));
        in = off <= bx->hi[a] - bx->lo[a];
      } else {
        in = x[a] >= bx->lo[a] && x[a] <= bx->hi[a];
      }
    }
    if (in) return 1;
  }
  return 0;
}
static int64_t box_lin(const olevel *L, const int64_t x[3], const int64_t lo[3], const int64_t n[3]) {
  (void)L;
  int64_t p[3];
  for (int a = 0; a < 3; ++a) {
    p[a] = x[a] - lo[a];
    if (p[a] < 0 || p[a] >= n[a]) return -1;
  }
  return p[0] + n[0] * (p[1] + n[1] * p[2]);
}
/* node id of canonical position x at level l, -1 if absent */
static int64_t node_id(const ora_t *o, int l, const int64_t x[3]) {
  const olevel *L = &o->lev[l];
  int64_t k = box_lin(L, x, L->blo, L->bn);
  return k < 0 ? -1 : L->id[k];
}
/* Chebyshev distance (fine units, capped at 3) of a canonical in-domain position to
 * the in-domain complement of the level-l region; 255 when outside the region.
 * Level 0 has no parent interface: 3. */
static int dist_at(const ora_t *o, int l, const int64_t x[3]) {
  if (l == 0) return 3;
  const olevel *L = &o->lev[l];
  int64_t p[3];
  for (int a = 0; a < 3; ++a) {
    p[a] = L->efull[a] ? x[a] : x[a] - L->elo[a];
    if (p[a] < 0 || p[a] >= L->en[a]) return 255;
  }
  return L->dist[p[0] + L->en[0] * (p[1] + L->en[1] * p[2])];
}

ora_t *ora_create(int D, const int64_t N[3], const int periodic[3], double nu0, int n_levels) {
  if (D != 2 && D != 3) return NULL;
  if (n_levels < 1 || n_levels > OMAXL) return NULL;
  ora_t *o = (ora_t *)calloc(1, sizeof(ora_t));
  o->D = D;
  o->Q = D == 2 ? 9 : 27;
  o->L = n_levels;
  for (int a = 0; a < 3; ++a) {
    o->N[a] = a < D ? N[a] : 1;
    o->periodic[a] = a < D ? (periodic[a] != 0) : 0;
  }
  for (int f = 0; f < 6; ++f) o->face_kind[f] = (f / 2 < D && !o->periodic[f / 2]) ? ORA_FACE_WALL : ORA_FACE_PERIODIC;
  o->nu0 = nu0;
  lattice(D, o->c, o->W);
  return o;
}

void ora_destroy(ora_t *o) {
  if (!o) return;
  for (int l = 0; l < OMAXL; ++l) {
    olevel *L = &o->lev[l];
    free(L->box);
    for (int s = 0; s < L->nsol; ++s) free(L->sol[s].mask);
    free(L->sol);
    free(L->dist);
    free(L->id);
    free(L->pos);
    free(L->solid);
    free(L->pd);
    free(L->ring);
    free(L->w);
    free(L->f);
    free(L->g);
    free(L->gam);
    free(L->force);
    free(L->vf);
    free(L->vg);
    free(L->lf);
    free(L->lg);
    free(L->lF);
  }
  for (int t = 0; t < o->ntape; ++t) {
    free(o->tape[t].g0);
    free(o->tape[t].g1);
  }
  free(o->tape);
  free(o);
}

const char *ora_error(const ora_t *o) { return o ? o->err : "null oracle"; }

int ora_set_face(ora_t *o, int face, int kind, const double u[3]) {
  if (o->finalized) return fail(o, -2, "set_face after finalize");
  if (face < 0 || face >= 6 || face / 2 >= o->D) return fail(o, -1, "bad face %d", face);
  if (o->periodic[face / 2]) return fail(o, -1, "face %d is on a periodic axis", face);
  if (kind < ORA_FACE_WALL || kind > ORA_FACE_OUTFLOW) return fail(o, -1, "bad face kind %d", kind);
  o->face_kind[face] = kind;
  for (int a = 0; a < 3; ++a) o->face_u[face][a] = u ? u[a] : 0.0;
  return 0;
}

int ora_add_box(ora_t *o, int l, const int64_t lo[3], const int64_t hi[3]) {
  if (o->finalized) return fail(o, -2, "add_box after finalize");
  if (l < 1 || l >= o->L) return fail(o, -1, "boxes are given for levels 1..L-1 (got %d)", l);
  obox b;
  for (int a = 0; a < 3; ++a) {
    b.lo[a] = a < o->D ? lo[a] : 0;
    b.hi[a] = a < o->D ? hi[a] : 0;
  }
  for (int a = 0; a < o->D; ++a) {
    if (b.hi[a] < b.lo[a]) return fail(o, -1, "empty box on axis %d", a);
    if (o->periodic[a]) {
      int64_t P = lv_period(o, l, a);
      if (b.lo[a] < 0 || b.lo[a] >= P || b.hi[a] - b.lo[a] > P - 1)
        return fail(o, -1, "box out of periodic range on axis %d", a);
      if (b.hi[a] - b.lo[a] == P - 1) continue;
    } else {
      if (b.lo[a] < 0 || b.hi[a] > lv_extent(o, l, a) - 1)
        return fail(o, -1, "box outside the domain on axis %d", a);
    }
    if ((b.lo[a] & 1) || (b.hi[a] & 1)) return fail(o, -1, "box faces must lie on parent nodes (axis %d)", a);
  }
  olevel *L = &o->lev[l];
  L->box = (obox *)realloc(L->box, sizeof(obox) * (L->nbox + 1));
  L->box[L->nbox++] = b;
  return 0;
}

int ora_set_solid(ora_t *o, int l, const int64_t lo[3], const int64_t n[3], const uint8_t *mask) {
  if (o->finalized) return fail(o, -2, "set_solid after finalize");
  if (l < 0 || l >= o->L) return fail(o, -1, "bad level");
  olevel *L = &o->lev[l];
  osolid s;
  int64_t tot = 1;
  for (int a = 0; a < 3; ++a) {
    s.lo[a] = a < o->D ? lo[a] : 0;
    s.n[a] = a < o->D ? n[a] : 1;
    if (s.n[a] < 1) return fail(o, -1, "bad solid extent");
    tot *= s.n[a];
  }
  s.mask = (uint8_t *)malloc((size_t)tot);
  memcpy(s.mask, mask, (size_t)tot);
  L->sol = (osolid *)realloc(L->sol, sizeof(osolid) * (L->nsol + 1));
  L->sol[L->nsol++] = s;
  return 0;
}

int ora_set_force_uniform(ora_t *o, const double F[3]) {
  for (int a = 0; a < 3; ++a) o->Fu[a] = a < o->D ? F[a] : 0.0;
  return 0;
}

/* index box of a level (a public convention): level 0 = whole domain; level l>0:
 * per axis the hull of its boxes, or the whole period when a box spans or wraps it */
static void make_index_box(ora_t *o, int l) {
  olevel *L = &o->lev[l];
  for (int a = 0; a < 3; ++a) {
    if (a >= o->D) {
      L->blo[a] = 0;
      L->bn[a] = 1;
      continue;
    }
    if (l == 0) {
      L->blo[a] = 0;
      L->bn[a] = lv_extent(o, 0, a);
      continue;
    }
    int64_t mn = INT64_MAX, mx = INT64_MIN;
    int whole = 0;
    for (int b = 0; b < L->nbox; ++b) {
      const obox *bx = &L->box[b];
      if (o->periodic[a] && (box_full(o, l, bx, a) || bx->hi[a] >= lv_period(o, l, a))) whole = 1;
      if (bx->lo[a] < mn) mn = bx->lo[a];
      if (bx->hi[a] > mx) mx = bx->hi[a];
    }
    if (whole) {
      L->blo[a] = 0;
      L->bn[a] = lv_period(o, l, a);
    } else {
      L->blo[a] = mn;
      L->bn[a] = mx - mn + 1;
    }
  }
}

/* distance grid by repeated erosion with the 3^D cube; out-of-domain positions do
 * not erode (faces on walls or spanning periodic axes carry no interface) */
static int make_dist(ora_t *o, int l) {
  olevel *L = &o->lev[l];
  int64_t tot = 1;
  for (int a = 0; a < 3; ++a) {
    if (a >= o->D) {
      L->elo[a] = 0;
      L->en[a] = 1;
      L->efull[a] = 0;
    } else if (o->periodic[a] && L->bn[a] == lv_period(o, l, a)) {
      L->elo[a] = 0;
      L->en[a] = L->bn[a];
      L->efull[a] = 1;
    } else {
      L->elo[a] = L->blo[a] - EXT_MARGIN;
      L->en[a] = L->bn[a] + 2 * EXT_MARGIN;
      L->efull[a] = 0;
    }
    tot *= L->en[a];
  }
  uint8_t *cur = (uint8_t *)malloc((size_t)tot), *nxt = (uint8_t *)malloc((size_t)tot);
  uint8_t *isreg = (uint8_t *)malloc((size_t)tot), *ood = (uint8_t *)malloc((size_t)tot);
  L->dist = (uint8_t *)malloc((size_t)tot);
  for (int64_t z = 0; z < L->en[2]; ++z)
    for (int64_t y = 0; y < L->en[1]; ++y)
      for (int64_t x = 0; x < L->en[0]; ++x) {
        int64_t k = x + L->en[0] * (y + L->en[1] * z);
        int64_t p[3] = {x + L->elo[0], y + L->elo[1], z + L->elo[2]};
        if (!canon(o, l, p)) {
          cur[k] = 1; /* out of domain: ignored, never eroded */
          isreg[k] = 0;
          ood[k] = 1;
        } else {
          cur[k] = (uint8_t)in_region(o, l, p);
          isreg[k] = cur[k];
          ood[k] = 0;
        }
        L->dist[k] = isreg[k] ? 0 : 255;
      }
  for (int it = 1; it <= 3; ++it) {
    for (int64_t z = 0; z < L->en[2]; ++z)
      for (int64_t y = 0; y < L->en[1]; ++y)
        for (int64_t x = 0; x < L->en[0]; ++x) {
          int64_t k = x + L->en[0] * (y + L->en[1] * z);
          if (ood[k]) {
            nxt[k] = 1;
            continue;
          }
          uint8_t v = cur[k];
          for (int dz = (o->D == 3 ? -1 : 0); dz <= (o->D == 3 ? 1 : 0) && v; ++dz)
            for (int dy = -1; dy <= 1 && v; ++dy)
              for (int dx = -1; dx <= 1 && v; ++dx) {
                int64_t q[3] = {x + dx, y + dy, z + dz};
                int ok = 1;
                for (int a = 0; a < 3; ++a) {
                  if (q[a] < 0 || q[a] >= L->en[a]) {
                    if (L->efull[a]) q[a] = wrapi(q[a], L->en[a]);
                    else ok = 0;
                  }
                }
                if (!ok) {
                  v = 0;
                  break;
                }
                v = cur[q[0] + L->en[0] * (q[1] + L->en[1] * q[2])];
              }
          nxt[k] = v;
        }
    for (int64_t k = 0; k < tot; ++k)
      if (isreg[k] && nxt[k]) L->dist[k] = (uint8_t)it;
    uint8_t *t = cur;
    cur = nxt;
    nxt = t;
  }
  free(cur);
  free(nxt);
  free(isreg);
  free(ood);
  return 0;
}

int ora_finalize(ora_t *o) {
  if (o->finalized) return fail(o, -2, "finalize twice");
  for (int l = 1; l < o->L; ++l)
    if (o->lev[l].nbox == 0) return fail(o, -1, "level %d has no boxes", l);
  for (int l = 0; l < o->L; ++l) {
    make_index_box(o, l);
    make_dist(o, l);
  }
  for (int l = 0; l < o->L; ++l) {
    olevel *L = &o->lev[l];
    int64_t tot = L->bn[0] * L->bn[1] * L->bn[2];
    L->id = (int32_t *)malloc(sizeof(int32_t) * (size_t)tot);
    int64_t nn = 0;
    for (int64_t k = 0; k < tot; ++k) {
      int64_t x[3] = {L->blo[0] + k % L->bn[0], L->blo[1] + (k / L->bn[0]) % L->bn[1],
                      L->blo[2] + k / (L->bn[0] * L->bn[1])};
      int exists = 0;
      int64_t xc[3] = {x[0], x[1], x[2]};
      if (canon(o, l, xc) && in_region(o, l, xc)) {
        exists = 1;
        if (l + 1 < o->L) {
          int64_t y[3] = {2 * xc[0], 2 * xc[1], 2 * xc[2]};
          if (canon(o, l + 1, y) && in_region(o, l + 1, y) && dist_at(o, l + 1, y) >= 3) exists = 0;
        }
      }
      L->id[k] = exists ? (int32_t)nn++ : -1;
    }
    L->nn = nn;
    L->pos = (int64_t *)malloc(sizeof(int64_t) * 3 * (size_t)(nn ? nn : 1));
    L->solid = (uint8_t *)calloc((size_t)(nn ? nn : 1), 1);
    L->pd = (uint8_t *)calloc((size_t)(nn ? nn : 1), 1);
    L->ring = (uint8_t *)calloc((size_t)(nn ? nn : 1), 1);
    for (int64_t k = 0; k < tot; ++k) {
      if (L->id[k] < 0) continue;
      int64_t n = L->id[k];
      int64_t x[3] = {L->blo[0] + k % L->bn[0], L->blo[1] + (k / L->bn[0]) % L->bn[1],
                      L->blo[2] + k / (L->bn[0] * L->bn[1])};
      for (int a = 0; a < 3; ++a) L->pos[3 * n + a] = x[a];
      int d = dist_at(o, l, x);
      L->pd[n] = (uint8_t)(d > 3 ? 3 : d);
      if (l + 1 < o->L) {
        int64_t y[3] = {2 * x[0], 2 * x[1], 2 * x[2]};
        if (canon(o, l + 1, y) && in_region(o, l + 1, y) && dist_at(o, l + 1, y) == 2) L->ring[n] = 1;
      }
      if (L->ring[n] && L->pd[n] < 2)
        return fail(o, -1, "level %d node (%lld,%lld,%lld) is both a ring node and a parent-interface node", l,
                    (long long)x[0], (long long)x[1], (long long)x[2]);
    }
    /* solids */
    for (int s = 0; s < L->nsol; ++s) {
      const osolid *S = &L->sol[s];
      for (int64_t z = 0; z < S->n[2]; ++z)
        for (int64_t y = 0; y < S->n[1]; ++y)
          for (int64_t x = 0; x < S->n[0]; ++x) {
            if (!S->mask[x + S->n[0] * (y + S->n[1] * z)]) continue;
            int64_t p[3] = {S->lo[0] + x, S->lo[1] + y, S->lo[2] + z};
            if (!canon(o, l, p)) return fail(o, -1, "solid node outside the domain");
            int64_t n = node_id(o, l, p);
            if (n < 0) return fail(o, -1, "solid node at a position with no level-%d node", l);
            if (L->pd[n] < 2 || L->ring[n]) return fail(o, -1, "solid node on an interface layer");
            L->solid[n] = 1;
          }
    }
    L->beta = ora_beta(o->nu0 * (double)(1 << l));
    L->f = (double *)calloc((size_t)(nn ? nn : 1) * o->Q, sizeof(double));
    L->g = (double *)calloc((size_t)(nn ? nn : 1) * o->Q, sizeof(double));
    L->vf = (uint8_t *)calloc((size_t)(nn ? nn : 1), 1);
    L->vg = (uint8_t *)calloc((size_t)(nn ? nn : 1) * o->Q, 1);
    L->gam = (double *)calloc((size_t)(nn ? nn : 1), sizeof(double));
    L->w = (double *)calloc((size_t)(nn ? nn : 1), sizeof(double));
  }
  /* owned-volume weights (reading R11).  The child owns the region R eroded by one
   * fine spacing; a node's cell is split into 2^D sub-cells, and sub-cell sigma of node
   * x lies in the owned part exactly when every fine node of the 4^D block spanning
   * [x-1, x+2] (sigma=+1) or [x-2, x+1] (sigma=-1) per axis is in R (out-of-domain
   * positions ignored).  Parent ring nodes own nothing. */
  for (int l = 0; l < o->L; ++l) {
    olevel *L = &o->lev[l];
    double base = 1.0;
    for (int a = 0; a < o->D; ++a) base /= (double)(1 << l);
    for (int64_t n = 0; n < L->nn; ++n) {
      if (L->solid[n] || L->ring[n]) {
        L->w[n] = 0.0;
        continue;
      }
      if (l == 0 || L->pd[n] >= 2) {
        L->w[n] = base;
        continue;
      }
      int cnt = 0, tot = 1 << o->D;
      for (int s = 0; s < tot; ++s) {
        int64_t a0[3] = {0, 0, 0}, a1[3] = {0, 0, 0};
        for (int a = 0; a < o->D; ++a) {
          int plus = (s >> a) & 1;
          a0[a] = L->pos[3 * n + a] + (plus ? -1 : -2);
          a1[a] = L->pos[3 * n + a] + (plus ? 2 : 1);
        }
        int ok = 1;
        for (int64_t z = a0[2]; z <= a1[2] && ok; ++z)
          for (int64_t y = a0[1]; y <= a1[1] && ok; ++y)
            for (int64_t x = a0[0]; x <= a1[0] && ok; ++x) {
              int64_t p[3] = {x, y, z};
              if (canon(o, l, p) && !in_region(o, l, p)) ok = 0;
            }
        cnt += ok;
      }
      L->w[n] = base * (double)cnt / (double)tot;
    }
  }
  o->finalized = 1;
  return 0;
}

int ora_level_box(const ora_t *o, int l, int64_t lo[3], int64_t n[3]) {
  if (!o->finalized || l < 0 || l >= o->L) return -1;
  for (int a = 0; a < 3; ++a) {
    lo[a] = o->lev[l].blo[a];
    n[a] = o->lev[l].bn[a];
  }
  return 0;
}

int ora_level_info(const ora_t *o, int l, int64_t *n_nodes, int64_t *n_fluid, double *beta) {
  if (!o->finalized || l < 0 || l >= o->L) return -1;
  const olevel *L = &o->lev[l];
  int64_t fl = 0;
  for (int64_t n = 0; n < L->nn; ++n) fl += !L->solid[n];
  if (n_nodes) *n_nodes = L->nn;
  if (n_fluid) *n_fluid = fl;
  if (beta) *beta = L->beta;
  return 0;
}

/* dense class map: -1 absent; else bit0 solid, bit1 ring, bits 2-3 parent distance (0..3) */
int ora_node_class(const ora_t *o, int l, int32_t *out) {
  if (!o->finalized || l < 0 || l >= o->L) return -1;
  const olevel *L = &o->lev[l];
  int64_t tot = L->bn[0] * L->bn[1] * L->bn[2];
  for (int64_t k = 0; k < tot; ++k) {
    int32_t n = L->id[k];
    out[k] = n < 0 ? -1 : (L->solid[n] | (L->ring[n] << 1) | (L->pd[n] << 2));
  }
  return 0;
}

int ora_weights(const ora_t *o, int l, double *out) {
  if (!o->finalized || l < 0 || l >= o->L) return -1;
  const olevel *L = &o->lev[l];
  int64_t tot = L->bn[0] * L->bn[1] * L->bn[2];
  for (int64_t k = 0; k < tot; ++k) out[k] = L->id[k] < 0 ? 0.0 : L->w[L->id[k]];
  return 0;
}

/* initial state: f_i = f^eq_i(rho, u) (1 + noise_i) at every fluid node; the state
 * is taken as complete on all levels at t0 (Sec. III.C, before step 1) */
int ora_init(ora_t *o, int l, const double *rho, const double *u, const double *noise) {
  if (!o->finalized) return fail(o, -2, "init before finalize");
  if (l < 0 || l >= o->L) return fail(o, -1, "bad level");
  olevel *L = &o->lev[l];
  int64_t tot = L->bn[0] * L->bn[1] * L->bn[2];
  for (int64_t k = 0; k < tot; ++k) {
    int32_t n = L->id[k];
    if (n < 0) continue;
    if (L->solid[n]) {
      L->vf[n] = 0;
      continue;
    }
    double uu[3] = {0, 0, 0};
    for (int a = 0; a < o->D; ++a) uu[a] = u[a * tot + k];
    ora_feq(o->D, rho[k], uu, &L->f[(size_t)n * o->Q]);
    if (noise)
      for (int i = 0; i < o->Q; ++i) L->f[(size_t)n * o->Q + i] *= 1.0 + noise[i * tot + k];
    L->vf[n] = 1;
    L->gam[n] = 2.0;
  }
  return 0;
}

int ora_set_f(ora_t *o, int l, const double *f) {
  if (!o->finalized || l < 0 || l >= o->L) return fail(o, -1, "bad level");
  olevel *L = &o->lev[l];
  int64_t tot = L->bn[0] * L->bn[1] * L->bn[2];
  for (int64_t k = 0; k < tot; ++k) {
    int32_t n = L->id[k];
    if (n < 0 || L->solid[n]) continue;
    for (int i = 0; i < o->Q; ++i) L->f[(size_t)n * o->Q + i] = f[i * tot + k];
    L->vf[n] = 1;
  }
  return 0;
}

int ora_set_force_field(ora_t *o, int l, const double *F) {
  if (!o->finalized || l < 0 || l >= o->L) return fail(o, -1, "bad level");
  olevel *L = &o->lev[l];
  int64_t tot = L->bn[0] * L->bn[1] * L->bn[2];
  if (!L->force) L->force = (double *)calloc((size_t)(L->nn ? L->nn : 1) * 3, sizeof(double));
  for (int64_t k = 0; k < tot; ++k) {
    int32_t n = L->id[k];
    if (n < 0) continue;
    for (int a = 0; a < o->D; ++a) L->force[3 * n + a] = F[a * tot + k];
  }
  return 0;
}

/* force density of node n in level-l units: forcing rescale du_f = du_c / r (Sec. III.A) */
static void node_force(const ora_t *o, int l, int64_t n, double F[3]) {
  const olevel *L = &o->lev[l];
  double s = 1.0 / (double)(1 << l);
  for (int a = 0; a < 3; ++a) {
    double v = o->Fu[a];
    if (L->force) v += L->force[3 * n + a];
    F[a] = v * s;
  }
}

/* ---------------------------------------------------------------------------
 * Streaming (left-hand side of Eq. f_equations): f_i(x) <- f'_i(x - c_i).
 * Boundary readings R9; a source that has no node at this level leaves the
 * population missing (valid bit 0).
 * ------------------------------------------------------------------------- */
enum { SRC_NODE = 0, SRC_BB = 1, SRC_INLET = 2, SRC_NONE = 3 };

/* where population i of node n of level l comes from when streaming: a node m
 * (SRC_NODE), the node's own opposite population (SRC_BB), the inlet equilibrium
 * (SRC_INLET, face in *face) or nowhere (SRC_NONE: no node at this level) */
static int stream_source(const ora_t *o, int l, int64_t n, int i, int64_t *m_out, int *face) {
  const olevel *L = &o->lev[l];
  int64_t y[3];
  int kind = SRC_NODE;
  for (int a = 0; a < 3; ++a) y[a] = L->pos[3 * n + a] - o->c[i][a];
  for (int a = 0; a < o->D; ++a) {
    if (o->periodic[a]) continue;
    int fc = -1;
    if (y[a] < 0) fc = 2 * a;
    else if (y[a] > lv_extent(o, l, a) - 1) fc = 2 * a + 1;
    if (fc < 0) continue;
    int fk = o->face_kind[fc];
    if (fk == ORA_FACE_WALL) kind = SRC_BB;
    else if (fk == ORA_FACE_INLET && kind != SRC_BB) {
      kind = SRC_INLET;
      *face = fc;
    } else if (fk == ORA_FACE_OUTFLOW) {
      y[a] += (fc & 1) ? -1 : 1; /* zero-gradient: take the value one node upstream */
    }
  }
  if (kind != SRC_NODE) return kind;
  if (!canon(o, l, y)) return SRC_NONE;
  int64_t m = node_id(o, l, y);
  if (m < 0) return SRC_NONE;
  if (L->solid[m]) return SRC_BB;
  *m_out = m;
  return SRC_NODE;
}

static double *dup_arr(const double *a, size_t n) {
  double *b = (double *)malloc(sizeof(double) * (n ? n : 1));
  memcpy(b, a, sizeof(double) * n);
  return b;
}
static void tape_push(ora_t *o, int op, int l, int skip) {
  if (!o->taping) return;
  if (o->ntape == o->captape) {
    o->captape = o->captape ? 2 * o->captape : 64;
    o->tape = (otape *)realloc(o->tape, sizeof(otape) * o->captape);
  }
  otape *t = &o->tape[o->ntape++];
  t->op = op;
  t->level = l;
  t->skip = skip;
  t->g0 = t->g1 = NULL;
  if (op == 1) t->g0 = dup_arr(o->lev[l].g, (size_t)o->lev[l].nn * o->Q);
  if (op == 2) {
    t->g0 = dup_arr(o->lev[l].g, (size_t)o->lev[l].nn * o->Q);
    t->g1 = dup_arr(o->lev[l + 1].g, (size_t)o->lev[l + 1].nn * o->Q);
  }
}
static void tape_clear(ora_t *o) {
  for (int t = 0; t < o->ntape; ++t) {
    free(o->tape[t].g0);
    free(o->tape[t].g1);
  }
  o->ntape = 0;
}

static void stream_level(ora_t *o, int l) {
  olevel *L = &o->lev[l];
  int Q = o->Q;
  tape_push(o, 0, l, 0);
  /* every node writes only its own post-stream populations: the node loop may run on
   * several threads (built with OpenMP) with identical results */
#pragma omp parallel for schedule(static)
  for (int64_t n = 0; n < L->nn; ++n) {
    if (L->solid[n]) continue;
    for (int i = 0; i < Q; ++i) {
      int64_t m = -1;
      int face = -1;
      int kind = stream_source(o, l, n, i, &m, &face);
      double val = NAN;
      uint8_t valid = 0;
      if (kind == SRC_NODE) {
        val = L->f[(size_t)m * Q + i];
        valid = L->vf[m];
      } else if (kind == SRC_BB) {
        val = L->f[(size_t)n * Q + (Q - 1 - i)];
        valid = L->vf[n];
      } else if (kind == SRC_INLET) {
        double feq[OMAXQ];
        ora_feq(o->D, 1.0, o->face_u[face], feq);
        val = feq[i];
        valid = 1;
      }
      L->g[(size_t)n * Q + i] = val;
      L->vg[(size_t)n * Q + i] = valid;
    }
  }
}

/* collision of one level (right-hand side of Eq. f_equations); skip_outer leaves the
 * outer interface layer uncollided (Sec. III.C step 1).  Every collided node must have
 * all populations present. */
/* population i of node n leaves towards a solid node (a bounce-back link) */
static int solid_link(const ora_t *o, int l, int64_t n, int i) {
  const olevel *L = &o->lev[l];
  int64_t y[3];
  for (int a = 0; a < 3; ++a) y[a] = L->pos[3 * n + a] + o->c[i][a];
  if (!canon(o, l, y)) return 0;
  int64_t m = node_id(o, l, y);
  return m >= 0 && L->solid[m];
}

static int collide_level(ora_t *o, int l, int skip_outer) {
  olevel *L = &o->lev[l];
  int Q = o->Q;
  tape_push(o, 1, l, skip_outer);
  /* per node: 0 collided, 1 skipped, 2 collided with a solid link, 3 missing input */
  uint8_t *st = (uint8_t *)malloc((size_t)(L->nn ? L->nn : 1));
  /* the collisions are independent per node (several threads when built with OpenMP);
   * the momentum-exchange sum below stays serial, in node order */
#pragma omp parallel for schedule(static)
  for (int64_t n = 0; n < L->nn; ++n) {
    st[n] = 1;
    if (L->solid[n]) continue;
    if (skip_outer && L->pd[n] == 0) {
      L->vf[n] = 0;
      continue;
    }
    int complete = 1;
    for (int i = 0; i < Q; ++i)
      if (!L->vg[(size_t)n * Q + i]) complete = 0;
    if (!complete) {
      st[n] = 3;
      continue;
    }
    double F[3];
    node_force(o, l, n, F);
    L->gam[n] = ora_kbc(o->D, L->beta, &L->g[(size_t)n * Q], F, &L->f[(size_t)n * Q], NULL, NULL);
    L->vf[n] = 1;
    st[n] = 0;
    for (int i = 0; i < Q; ++i)
      if (solid_link(o, l, n, i)) st[n] = 2;
  }
  for (int64_t n = 0; n < L->nn; ++n)
    if (st[n] == 3) {
      int i = 0;
      while (i < Q && L->vg[(size_t)n * Q + i]) ++i;
      free(st);
      return fail(o, -10, "level %d node (%lld,%lld,%lld) collides with missing population %d", l,
                  (long long)L->pos[3 * n], (long long)L->pos[3 * n + 1], (long long)L->pos[3 * n + 2], i);
    }
  /* momentum exchange on links into solid nodes (reading R10), from the post-collision
   * populations of this step */
  double step_drag[3] = {0, 0, 0};
  for (int64_t n = 0; n < L->nn; ++n) {
    if (st[n] != 2) continue;
    for (int i = 0; i < Q; ++i)
      if (solid_link(o, l, n, i))
        for (int a = 0; a < 3; ++a) step_drag[a] += 2.0 * o->c[i][a] * L->f[(size_t)n * Q + i];
  }
  free(st);
  for (int a = 0; a < 3; ++a) L->drag[a] += step_drag[a];
  L->drag_steps++;
  return 0;
}

/* post-stream macroscopic values and non-equilibrium part at one node */
static void node_macro(const ora_t *o, const double *g, double *rho, double u[3], double *fneq) {
  int Q = o->Q;
  double r = 0, j[3] = {0, 0, 0};
  for (int i = 0; i < Q; ++i) {
    r += g[i];
    for (int a = 0; a < 3; ++a) j[a] += o->c[i][a] * g[i];
  }
  for (int a = 0; a < 3; ++a) u[a] = j[a] / r;
  *rho = r;
  double feq[OMAXQ];
  ora_feq(o->D, r, u, feq);
  for (int i = 0; i < Q; ++i) fneq[i] = g[i] - feq[i];
}

static int node_complete(const ora_t *o, const olevel *L, int64_t n) {
  for (int i = 0; i < o->Q; ++i)
    if (!L->vg[(size_t)n * o->Q + i]) return 0;
  return 1;
}

/* composite stencil value at a coarse-aligned position X (parent coordinates), at
 * child scale (reading R7; rescaling Eq. f_neq_rescaling_iso with r = 2) */
static int point_value(ora_t *o, int lp, const int64_t Xin[3], double *rho, double u[3], double *fneq) {
  olevel *P = &o->lev[lp], *C = &o->lev[lp + 1];
  int64_t X[3] = {Xin[0], Xin[1], Xin[2]};
  if (!canon(o, lp, X)) return fail(o, -11, "interpolation point outside the domain");
  int64_t xc[3] = {2 * X[0], 2 * X[1], 2 * X[2]};
  if (canon(o, lp + 1, xc) && in_region(o, lp + 1, xc) && dist_at(o, lp + 1, xc) >= 2) {
    int64_t m = node_id(o, lp + 1, xc);
    if (m < 0 || C->solid[m] || !node_complete(o, C, m))
      return fail(o, -12, "child stencil value missing at level %d (%lld,%lld,%lld)", lp + 1, (long long)xc[0],
                  (long long)xc[1], (long long)xc[2]);
    node_macro(o, &C->g[(size_t)m * o->Q], rho, u, fneq);
    return 0;
  }
  int64_t m = node_id(o, lp, X);
  if (m < 0 || P->solid[m] || P->ring[m] || !node_complete(o, P, m))
    return fail(o, -13, "parent stencil value missing at level %d (%lld,%lld,%lld)", lp, (long long)X[0],
                (long long)X[1], (long long)X[2]);
  node_macro(o, &P->g[(size_t)m * o->Q], rho, u, fneq);
  double fac = P->beta / (2.0 * C->beta);
  for (int i = 0; i < o->Q; ++i) fneq[i] *= fac;
  return 0;
}

/* Sec. III.C steps 3-4 for the pair (lp, lp+1) at the common time instant:
 * rescale twin nodes both ways and reconstruct the hanging fine nodes. */
static int couple(ora_t *o, int lp) {
  olevel *P = &o->lev[lp], *C = &o->lev[lp + 1];
  int Q = o->Q, D = o->D;
  tape_push(o, 2, lp, 0);
  /* new child interface states, computed from the unmodified post-stream fields */
  double *newc = (double *)malloc(sizeof(double) * (size_t)(C->nn ? C->nn : 1) * Q);
  uint8_t *setc = (uint8_t *)calloc((size_t)(C->nn ? C->nn : 1), 1);
  double *newp = (double *)malloc(sizeof(double) * (size_t)(P->nn ? P->nn : 1) * Q);
  uint8_t *setp = (uint8_t *)calloc((size_t)(P->nn ? P->nn : 1), 1);
  int rc = 0;
  static const double w4[4] = {-1.0 / 16.0, 9.0 / 16.0, 9.0 / 16.0, -1.0 / 16.0};
  /* error code per child node; the nodes are independent (several threads when built
   * with OpenMP), the first error in node order is returned */
  int *crc = (int *)calloc((size_t)(C->nn ? C->nn : 1), sizeof(int));
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t n = 0; n < C->nn; ++n) {
    if (C->solid[n] || C->pd[n] > 1) continue;
    int rc = 0;
    const int64_t *x = &C->pos[3 * n];
    int npt[3] = {1, 1, 1};
    int64_t pts[3][4];
    double wts[3][4];
    for (int a = 0; a < 3; ++a) {
      if (a < D && (x[a] & 1)) {
        /* Eq. interp with spacing = fine spacing: points x-3, x-1, x+1, x+3 (fine) */
        npt[a] = 4;
        for (int k = 0; k < 4; ++k) {
          pts[a][k] = (x[a] - 3 + 2 * k) / 2; /* exact: x odd */
          wts[a][k] = w4[k];
        }
      } else {
        pts[a][0] = x[a] / 2;
        wts[a][0] = 1.0;
      }
    }
    double rr = 0, uu[3] = {0, 0, 0}, nn_[OMAXQ];
    for (int i = 0; i < Q; ++i) nn_[i] = 0.0;
    for (int kz = 0; kz < npt[2] && !rc; ++kz)
      for (int ky = 0; ky < npt[1] && !rc; ++ky)
        for (int kx = 0; kx < npt[0] && !rc; ++kx) {
          int64_t X[3] = {pts[0][kx], pts[1][ky], pts[2][kz]};
          double w = wts[0][kx] * wts[1][ky] * wts[2][kz];
          double r, u[3], fn[OMAXQ];
          rc = point_value(o, lp, X, &r, u, fn);
          if (rc) break;
          rr += w * r;
          for (int a = 0; a < 3; ++a) uu[a] += w * u[a];
          for (int i = 0; i < Q; ++i) nn_[i] += w * fn[i];
        }
    if (rc) {
      crc[n] = rc;
      continue;
    }
    double feq[OMAXQ];
    ora_feq(D, rr, uu, feq);
    for (int i = 0; i < Q; ++i) newc[(size_t)n * Q + i] = feq[i] + nn_[i];
    setc[n] = 1;
  }
  for (int64_t n = 0; n < C->nn && !rc; ++n) rc = crc[n];
  free(crc);
  /* coarse ring nodes from co-located fine nodes (inverse of Eq. f_neq_rescaling_iso) */
  int *prc = (int *)calloc((size_t)(P->nn ? P->nn : 1), sizeof(int));
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t n = 0; n < P->nn; ++n) {
    if (rc || !P->ring[n]) continue;
    int64_t xc[3] = {2 * P->pos[3 * n], 2 * P->pos[3 * n + 1], 2 * P->pos[3 * n + 2]};
    int64_t m = node_id(o, lp + 1, xc);
    if (m < 0 || C->solid[m] || !node_complete(o, C, m)) {
      prc[n] = fail(o, -14, "fine twin of ring node missing at level %d", lp + 1);
      continue;
    }
    double r, u[3], fn[OMAXQ], feq[OMAXQ];
    node_macro(o, &C->g[(size_t)m * Q], &r, u, fn);
    ora_feq(D, r, u, feq);
    double fac = 2.0 * C->beta / P->beta;
    for (int i = 0; i < Q; ++i) newp[(size_t)n * Q + i] = feq[i] + fac * fn[i];
    setp[n] = 1;
  }
  for (int64_t n = 0; n < P->nn && !rc; ++n) rc = prc[n];
  free(prc);
  if (!rc) {
    for (int64_t n = 0; n < C->nn; ++n)
      if (setc[n])
        for (int i = 0; i < Q; ++i) {
          C->g[(size_t)n * Q + i] = newc[(size_t)n * Q + i];
          C->vg[(size_t)n * Q + i] = 1;
        }
    for (int64_t n = 0; n < P->nn; ++n)
      if (setp[n])
        for (int i = 0; i < Q; ++i) {
          P->g[(size_t)n * Q + i] = newp[(size_t)n * Q + i];
          P->vg[(size_t)n * Q + i] = 1;
        }
  }
  free(newc);
  free(setc);
  free(newp);
  free(setp);
  return rc;
}

/* Sec. III.C steps 3-4 alone, for checking them in isolation: the post-stream states
 * of the pair (lp, lp+1) are taken from dense [Q][box] arrays (a non-finite value is a
 * missing population), coupled, and written back in place (the states after the
 * rescaling and reconstruction; populations still missing read NaN). */
int ora_couple_states(ora_t *o, int lp, double *gp, double *gc) {
  if (!o->finalized) return fail(o, -2, "couple before finalize");
  if (lp < 0 || lp + 1 >= o->L) return fail(o, -1, "bad parent level");
  double *arr[2] = {gp, gc};
  for (int s = 0; s < 2; ++s) {
    olevel *L = &o->lev[lp + s];
    int64_t tot = L->bn[0] * L->bn[1] * L->bn[2];
    for (int64_t k = 0; k < tot; ++k) {
      int32_t n = L->id[k];
      if (n < 0) continue;
      for (int i = 0; i < o->Q; ++i) {
        double v = arr[s][i * tot + k];
        L->g[(size_t)n * o->Q + i] = v;
        L->vg[(size_t)n * o->Q + i] = (uint8_t)(!L->solid[n] && isfinite(v));
      }
    }
  }
  int rc = couple(o, lp);
  if (rc) return rc;
  for (int s = 0; s < 2; ++s) {
    olevel *L = &o->lev[lp + s];
    int64_t tot = L->bn[0] * L->bn[1] * L->bn[2];
    for (int64_t k = 0; k < tot; ++k) {
      int32_t n = L->id[k];
      for (int i = 0; i < o->Q; ++i)
        arr[s][i * tot + k] = (n < 0 || !L->vg[(size_t)n * o->Q + i]) ? NAN : L->g[(size_t)n * o->Q + i];
    }
  }
  return 0;
}

/* Sec. III.C, applied recursively: the five steps for the pair (l, l+1) run inside
 * the advection of level l. */
static int cycle(ora_t *o, int l) {
  int rc;
  stream_level(o, l);
  if (l + 1 < o->L) {
    if ((rc = cycle(o, l + 1))) return rc;             /* step 1: first fine substep ... */
    if ((rc = collide_level(o, l + 1, 1))) return rc;  /* ... collide, outer layer skipped */
    if ((rc = cycle(o, l + 1))) return rc;             /* step 2: second fine advection */
    if ((rc = couple(o, l))) return rc;                /* steps 3-4 */
    if ((rc = collide_level(o, l + 1, 0))) return rc;  /* step 5 for the fine level */
  }
  return 0;
}

int ora_advance(ora_t *o, int steps) {
  if (!o->finalized) return fail(o, -2, "advance before finalize");
  for (int s = 0; s < steps; ++s) {
    int rc = cycle(o, 0);
    if (rc) return rc;
    rc = collide_level(o, 0, 0); /* step 5 for the coarsest level */
    if (rc) return rc;
  }
  return 0;
}

int ora_get_f(const ora_t *o, int l, double *out) {
  if (!o->finalized || l < 0 || l >= o->L) return -1;
  const olevel *L = &o->lev[l];
  int64_t tot = L->bn[0] * L->bn[1] * L->bn[2];
  for (int64_t k = 0; k < tot; ++k) {
    int32_t n = L->id[k];
    for (int i = 0; i < o->Q; ++i)
      out[i * tot + k] = (n < 0 || L->solid[n] || !L->vf[n]) ? NAN : L->f[(size_t)n * o->Q + i];
  }
  return 0;
}

/* macroscopic output from the stored post-collision state: rho = sum f',
 * u = sum c f'/rho - du/2 (equal to j/rho + du/2 before the collision, reading R8) */
int ora_moments(const ora_t *o, int l, double *rho, double *u, double *gamma) {
  if (!o->finalized || l < 0 || l >= o->L) return -1;
  const olevel *L = &o->lev[l];
  int64_t tot = L->bn[0] * L->bn[1] * L->bn[2];
  for (int64_t k = 0; k < tot; ++k) {
    int32_t n = L->id[k];
    if (n < 0 || L->solid[n] || !L->vf[n]) {
      if (rho) rho[k] = NAN;
      if (u)
        for (int a = 0; a < o->D; ++a) u[a * tot + k] = NAN;
      if (gamma) gamma[k] = NAN;
      continue;
    }
    double r = 0, j[3] = {0, 0, 0};
    for (int i = 0; i < o->Q; ++i) {
      double f = L->f[(size_t)n * o->Q + i];
      r += f;
      for (int a = 0; a < 3; ++a) j[a] += o->c[i][a] * f;
    }
    double F[3];
    node_force(o, l, n, F);
    if (rho) rho[k] = r;
    if (u)
      for (int a = 0; a < o->D; ++a) u[a * tot + k] = j[a] / r - 0.5 * F[a] / r;
    if (gamma) gamma[k] = L->gam[n];
  }
  return 0;
}

int ora_sample_f(const ora_t *o, int l, int64_t n, const int64_t *coords, double *out) {
  if (!o->finalized || l < 0 || l >= o->L) return -1;
  const olevel *L = &o->lev[l];
  for (int64_t s = 0; s < n; ++s) {
    int64_t x[3] = {coords[3 * s], coords[3 * s + 1], coords[3 * s + 2]};
    int64_t m = canon(o, l, x) ? node_id(o, l, x) : -1;
    for (int i = 0; i < o->Q; ++i)
      out[s * o->Q + i] = (m < 0 || L->solid[m] || !L->vf[m]) ? NAN : L->f[(size_t)m * o->Q + i];
  }
  return 0;
}

/* mass and momentum over owned volumes (reading R11), coarse volume units */
int ora_reduce(const ora_t *o, double *mass, double mom[3]) {
  if (!o->finalized) return -1;
  double M = 0, J[3] = {0, 0, 0};
  for (int l = 0; l < o->L; ++l) {
    const olevel *L = &o->lev[l];
    for (int64_t n = 0; n < L->nn; ++n) {
      if (L->w[n] == 0.0) continue;
      double r = 0, j[3] = {0, 0, 0};
      for (int i = 0; i < o->Q; ++i) {
        double f = L->f[(size_t)n * o->Q + i];
        r += f;
        for (int a = 0; a < 3; ++a) j[a] += o->c[i][a] * f;
      }
      double F[3];
      node_force(o, l, n, F);
      M += L->w[n] * r;
      for (int a = 0; a < 3; ++a) J[a] += L->w[n] * (j[a] - 0.5 * F[a]);
    }
  }
  *mass = M;
  for (int a = 0; a < 3; ++a) mom[a] = J[a];
  return 0;
}

int ora_drag(ora_t *o, int l, double F[3], int64_t *steps, int reset) {
  if (!o->finalized || l < 0 || l >= o->L) return -1;
  olevel *L = &o->lev[l];
  for (int a = 0; a < 3; ++a) F[a] = L->drag[a];
  if (steps) *steps = L->drag_steps;
  if (reset) {
    L->drag[0] = L->drag[1] = L->drag[2] = 0.0;
    L->drag_steps = 0;
  }
  return 0;
}

/* ===========================================================================
 * Re-meshing (adaptive refinement, proposed in Sec. V): the state of a lattice is
 * carried over to another lattice of the same domain, levels and parameters whose
 * refinement blocks differ, at a coarse-step boundary (every level holds a
 * post-collision state at the same time instant).  Reading R15, per node of the new
 * lattice:
 *   1. the old lattice has a node at the same level and position: its populations;
 *   2. else the old lattice has a node one level finer at the same position (the
 *      region was refined and no longer is): coalescence of that node;
 *   3. else (a newly refined region): reconstruction from the old lattice as in
 *      Eq. interp, with the composite values of reading R7 (old nodes of the same level
 *      where present, old parent nodes brought to the finer scale elsewhere).
 * Density and velocity are carried over exactly (1) or by the four-point
 * reconstruction (3); the non-equilibrium part of a post-collision state is
 * f' - f^eq = (1 - 2 beta)(f - f^eq) for the LBGK value gamma = 2 of resolved flow
 * (Eq. f_mirr), so Eq. f_neq_rescaling_iso becomes, for post-collision states, the
 * factor beta_c (1 - 2 beta_f) / (2 beta_f (1 - 2 beta_c)) from coarse to fine and its
 * inverse from fine to coarse.
 * ------------------------------------------------------------------------- */

/* rho, u and the non-equilibrium part of the stored post-collision state of node m */
static void state_macro(const ora_t *o, int l, int64_t m, double *rho, double u[3], double *fneq) {
  const olevel *L = &o->lev[l];
  double r = 0, j[3] = {0, 0, 0};
  for (int i = 0; i < o->Q; ++i) {
    double f = L->f[(size_t)m * o->Q + i];
    r += f;
    for (int a = 0; a < 3; ++a) j[a] += o->c[i][a] * f;
  }
  for (int a = 0; a < 3; ++a) u[a] = j[a] / r;
  *rho = r;
  double feq[OMAXQ];
  ora_feq(o->D, r, u, feq);
  for (int i = 0; i < o->Q; ++i) fneq[i] = L->f[(size_t)m * o->Q + i] - feq[i];
}

/* post-collision non-equilibrium factor from level lc to level lc + 1 */
static double post_factor(const ora_t *o, int lc) {
  double bc = o->lev[lc].beta, bf = o->lev[lc + 1].beta;
  return bc * (1.0 - 2.0 * bf) / (2.0 * bf * (1.0 - 2.0 * bc));
}

/* fluid node of the old lattice at level l, canonical position x; -1 if none */
static int64_t old_node(const ora_t *s, int l, const int64_t xin[3]) {
  int64_t x[3] = {xin[0], xin[1], xin[2]};
  if (!canon(s, l, x)) return -1;
  int64_t m = node_id(s, l, x);
  if (m < 0 || s->lev[l].solid[m] || !s->lev[l].vf[m]) return -1;
  return m;
}

int ora_transfer_state(ora_t *d, const ora_t *s) {
  if (!d->finalized || !s->finalized) return fail(d, -2, "transfer before finalize");
  if (d->D != s->D || d->L != s->L || d->nu0 != s->nu0) return fail(d, -1, "transfer: lattices differ");
  for (int a = 0; a < 3; ++a)
    if (d->N[a] != s->N[a] || d->periodic[a] != s->periodic[a] || d->Fu[a] != s->Fu[a])
      return fail(d, -1, "transfer: domains differ");
  for (int f = 0; f < 6; ++f)
    if (d->face_kind[f] != s->face_kind[f]) return fail(d, -1, "transfer: boundaries differ");
  int Q = d->Q, D = d->D;
  static const double w4[4] = {-1.0 / 16.0, 9.0 / 16.0, 9.0 / 16.0, -1.0 / 16.0};
  for (int l = 0; l < d->L; ++l) {
    olevel *L = &d->lev[l];
    for (int64_t n = 0; n < L->nn; ++n) {
      L->vf[n] = 0;
      if (L->solid[n]) continue;
      const int64_t *x = &L->pos[3 * n];
      double *out = &L->f[(size_t)n * Q];
      int64_t xs[3] = {x[0], x[1], x[2]};
      int64_t m = old_node(s, l, xs);
      if (m >= 0) { /* 1. same node */
        memcpy(out, &s->lev[l].f[(size_t)m * Q], sizeof(double) * Q);
        L->gam[n] = s->lev[l].gam[m];
        L->vf[n] = 1;
        continue;
      }
      if (canon(s, l, xs)) {
        int64_t k = node_id(s, l, xs);
        if (k >= 0 && s->lev[l].solid[k]) return fail(d, -1, "transfer: level %d node solid in the old lattice only", l);
      }
      if (l + 1 < d->L) { /* 2. coalescence of the old finer node */
        int64_t xc[3] = {2 * x[0], 2 * x[1], 2 * x[2]};
        int64_t mc = old_node(s, l + 1, xc);
        if (mc >= 0) {
          double r, u[3], fn[OMAXQ], feq[OMAXQ];
          state_macro(s, l + 1, mc, &r, u, fn);
          ora_feq(D, r, u, feq);
          double fac = 1.0 / post_factor(s, l);
          for (int i = 0; i < Q; ++i) out[i] = feq[i] + fac * fn[i];
          L->gam[n] = 2.0;
          L->vf[n] = 1;
          continue;
        }
      }
      if (l == 0) return fail(d, -1, "transfer: no source for level 0 node");
      /* 3. reconstruction (Eq. interp) from composite old values at parent positions */
      int npt[3] = {1, 1, 1};
      int64_t pts[3][4];
      double wts[3][4];
      for (int a = 0; a < 3; ++a) {
        if (a < D && (x[a] & 1)) {
          npt[a] = 4;
          for (int k = 0; k < 4; ++k) {
            pts[a][k] = (x[a] - 3 + 2 * k) / 2;
            wts[a][k] = w4[k];
          }
        } else {
          pts[a][0] = x[a] / 2;
          wts[a][0] = 1.0;
        }
      }
      double rr = 0, uu[3] = {0, 0, 0}, nn_[OMAXQ];
      for (int i = 0; i < Q; ++i) nn_[i] = 0.0;
      for (int kz = 0; kz < npt[2]; ++kz)
        for (int ky = 0; ky < npt[1]; ++ky)
          for (int kx = 0; kx < npt[0]; ++kx) {
            int64_t X[3] = {pts[0][kx], pts[1][ky], pts[2][kz]};
            double w = wts[0][kx] * wts[1][ky] * wts[2][kz];
            double r, u[3], fn[OMAXQ];
            int64_t xf[3] = {2 * X[0], 2 * X[1], 2 * X[2]};
            int64_t mf = old_node(s, l, xf);
            if (mf >= 0) {
              state_macro(s, l, mf, &r, u, fn);
            } else {
              int64_t mp = old_node(s, l - 1, X);
              if (mp < 0)
                return fail(d, -1, "transfer: level %d node (%lld,%lld,%lld) has no source", l, (long long)x[0],
                            (long long)x[1], (long long)x[2]);
              state_macro(s, l - 1, mp, &r, u, fn);
              double fac = post_factor(s, l - 1);
              for (int i = 0; i < Q; ++i) fn[i] *= fac;
            }
            rr += w * r;
            for (int a = 0; a < 3; ++a) uu[a] += w * u[a];
            for (int i = 0; i < Q; ++i) nn_[i] += w * fn[i];
          }
      double feq[OMAXQ];
      ora_feq(D, rr, uu, feq);
      for (int i = 0; i < Q; ++i) out[i] = feq[i] + nn_[i];
      L->gam[n] = 2.0;
      L->vf[n] = 1;
    }
    L->drag[0] = L->drag[1] = L->drag[2] = 0.0;
    L->drag_steps = 0;
  }
  return 0;
}

/* ===========================================================================
 * Discrete adjoint (reverse mode of the exact forward map above, FP64).
 * The paper has no adjoint; this is the transpose of the linearisation of the
 * discrete coarse step defined by Sec. II.A and Sec. III.C as implemented here.
 * At nodes with <dh|dh> = 0 gamma is the constant 2 (reading R3), so dgamma/df = 0.
 * ========================================================================= */

/* d ln phi / du for the per-axis factor phi(c) = (2 - s) X^c of Eq. feq_iso,
 * s = sqrt(1 + 3u^2), X = (2u + s)/(1 - u) */
static double dlnphi(double u, int c) {
  double s = sqrt(1.0 + 3.0 * u * u), ds = 3.0 * u / s;
  double d = -ds / (2.0 - s);
  if (c) d += c * ((2.0 + ds) / (2.0 * u + s) + 1.0 / (1.0 - u));
  return d;
}

/* adjoint of f^eq(rho, u): given lam (adjoint of f^eq), accumulate into lrho, lu */
static void feq_T(int D, double rho, const double u[3], const double *lam, double *lrho, double lu[3]) {
  int c[OMAXQ][3];
  double W[OMAXQ], feq[OMAXQ];
  lattice(D, c, W);
  ora_feq(D, rho, u, feq);
  int Q = D == 2 ? 9 : 27;
  for (int i = 0; i < Q; ++i) {
    *lrho += lam[i] * feq[i] / rho;
    for (int a = 0; a < D; ++a) lu[a] += lam[i] * feq[i] * dlnphi(u[a], c[i][a]);
  }
}

/* S^T lam for the shear projection S (explicit matrix from unit vectors) */
static void shear_T(int D, const double *lam, double *out) {
  int c[OMAXQ][3];
  double W[OMAXQ];
  lattice(D, c, W);
  int Q = D == 2 ? 9 : 27;
  double e[OMAXQ], col[OMAXQ];
  for (int j = 0; j < Q; ++j) out[j] = 0.0;
  for (int j = 0; j < Q; ++j) {
    for (int k = 0; k < Q; ++k) e[k] = (k == j);
    shear_part(D, c, e, col); /* column j of S */
    for (int i = 0; i < Q; ++i) out[j] += col[i] * lam[i];
  }
}

/* reverse of ora_kbc: lo = adjoint of f'; returns adjoint of f (overwrites lf) and
 * adds the adjoint of the force density F to lF */
void ora_kbc_adj(int D, double beta, const double *f, const double F[3], const double *lo, double *lf,
                 double lF[3]) {
  int c[OMAXQ][3];
  double W[OMAXQ];
  lattice(D, c, W);
  int Q = D == 2 ? 9 : 27;
  double rho = 0, j[3] = {0, 0, 0};
  for (int i = 0; i < Q; ++i) {
    rho += f[i];
    for (int a = 0; a < 3; ++a) j[a] += c[i][a] * f[i];
  }
  double u[3] = {j[0] / rho, j[1] / rho, j[2] / rho};
  double feq[OMAXQ], d[OMAXQ], ds[OMAXQ], dh[OMAXQ];
  ora_feq(D, rho, u, feq);
  for (int i = 0; i < Q; ++i) d[i] = f[i] - feq[i];
  shear_part(D, c, d, ds);
  for (int i = 0; i < Q; ++i) dh[i] = d[i] - ds[i];
  double A = 0, B = 0;
  for (int i = 0; i < Q; ++i) {
    A += ds[i] * dh[i] / feq[i];
    B += dh[i] * dh[i] / feq[i];
  }
  double gamma = 2.0;
  int active = 0;
  if (B > 0.0) {
    double g = 1.0 / beta - (2.0 - 1.0 / beta) * A / B;
    if (isfinite(g)) {
      gamma = g;
      active = 1;
    }
  }
  double lds[OMAXQ], ldh[OMAXQ], lfeq[OMAXQ], ld[OMAXQ], tmp[OMAXQ];
  double lrho = 0, lu[3] = {0, 0, 0};
  for (int i = 0; i < Q; ++i) {
    lf[i] = lo[i];
    lds[i] = -2.0 * beta * lo[i];
    ldh[i] = -beta * gamma * lo[i];
    lfeq[i] = 0.0;
  }
  if (active) {
    double lg = 0;
    for (int i = 0; i < Q; ++i) lg += -beta * lo[i] * dh[i];
    double cc = 2.0 - 1.0 / beta;
    double lA = -cc / B * lg, lB = cc * A / (B * B) * lg;
    for (int i = 0; i < Q; ++i) {
      lds[i] += lA * dh[i] / feq[i];
      ldh[i] += lA * ds[i] / feq[i] + 2.0 * lB * dh[i] / feq[i];
      lfeq[i] += -(lA * ds[i] * dh[i] + lB * dh[i] * dh[i]) / (feq[i] * feq[i]);
    }
  }
  for (int i = 0; i < Q; ++i) {
    ld[i] = ldh[i];
    lds[i] -= ldh[i];
  }
  shear_T(D, lds, tmp);
  for (int i = 0; i < Q; ++i) ld[i] += tmp[i];
  for (int i = 0; i < Q; ++i) {
    lf[i] += ld[i];
    lfeq[i] -= ld[i];
  }
  /* the forcing term vanishes at F = 0 but its derivative does not: always reversed
   * when the force adjoint is requested */
  if (F && (lF || F[0] != 0.0 || F[1] != 0.0 || F[2] != 0.0)) {
    double v[3] = {u[0] + F[0] / rho, u[1] + F[1] / rho, u[2] + F[2] / rho};
    double lv[3] = {0, 0, 0};
    feq_T(D, rho, v, lo, &lrho, lv);
    for (int i = 0; i < Q; ++i) lfeq[i] -= lo[i];
    for (int a = 0; a < D; ++a) {
      lu[a] += lv[a];
      lrho -= lv[a] * F[a] / (rho * rho);
      if (lF) lF[a] += lv[a] / rho;
    }
  }
  feq_T(D, rho, u, lfeq, &lrho, lu);
  double lj[3] = {0, 0, 0};
  for (int a = 0; a < D; ++a) {
    lj[a] = lu[a] / rho;
    lrho -= lu[a] * u[a] / rho;
  }
  for (int i = 0; i < Q; ++i) {
    lf[i] += lrho;
    for (int a = 0; a < D; ++a) lf[i] += c[i][a] * lj[a];
  }
}

/* adjoint of (rho, u, fac (g - f^eq(rho, u))) with rho, u the moments of g:
 * accumulate into lg */
static void macro_T(const ora_t *o, const double *g, double fac, double lrho, const double lu_in[3],
                    const double *ln, double *lg) {
  int Q = o->Q, D = o->D;
  double rho = 0, j[3] = {0, 0, 0};
  for (int i = 0; i < Q; ++i) {
    rho += g[i];
    for (int a = 0; a < 3; ++a) j[a] += o->c[i][a] * g[i];
  }
  double u[3] = {j[0] / rho, j[1] / rho, j[2] / rho};
  double lfeq[OMAXQ] = {0}, lu[3] = {lu_in[0], lu_in[1], lu_in[2]};
  for (int i = 0; i < Q; ++i) {
    lg[i] += fac * ln[i];
    lfeq[i] = -fac * ln[i];
  }
  feq_T(D, rho, u, lfeq, &lrho, lu);
  double lj[3] = {0, 0, 0};
  for (int a = 0; a < D; ++a) {
    lj[a] = lu[a] / rho;
    lrho -= lu[a] * u[a] / rho;
  }
  for (int i = 0; i < Q; ++i) {
    lg[i] += lrho;
    for (int a = 0; a < D; ++a) lg[i] += o->c[i][a] * lj[a];
  }
}

/* reverse of stream_level: lf[source] += lg, then lg = 0 */
static void adj_stream(ora_t *o, int l) {
  olevel *L = &o->lev[l];
  int Q = o->Q;
  for (int64_t n = 0; n < L->nn; ++n) {
    if (L->solid[n]) continue;
    for (int i = 0; i < Q; ++i) {
      double v = L->lg[(size_t)n * Q + i];
      L->lg[(size_t)n * Q + i] = 0.0;
      if (v == 0.0) continue;
      int64_t m = -1;
      int face = -1;
      int kind = stream_source(o, l, n, i, &m, &face);
      if (kind == SRC_NODE) L->lf[(size_t)m * Q + i] += v;
      else if (kind == SRC_BB) L->lf[(size_t)n * Q + (Q - 1 - i)] += v;
    }
  }
}

typedef struct {
  int objective; /* 0: mean drag along dir on body_level, 1: final kinetic energy */
  int body_level;
  double dir[3];
  double nsub; /* number of body-level collisions in the run */
} oadj_obj;

/* reverse of collide_level with input snapshot g; adds the drag seed first */
static void adj_collide(ora_t *o, int l, int skip_outer, const double *g, const oadj_obj *ob) {
  olevel *L = &o->lev[l];
  int Q = o->Q;
  for (int64_t n = 0; n < L->nn; ++n) {
    if (L->solid[n]) continue;
    if (skip_outer && L->pd[n] == 0) continue;
    double *lo = &L->lf[(size_t)n * Q];
    if (ob->objective == 0 && l == ob->body_level) {
      for (int i = 0; i < Q; ++i) {
        int64_t y[3];
        for (int a = 0; a < 3; ++a) y[a] = L->pos[3 * n + a] + o->c[i][a];
        if (!canon(o, l, y)) continue;
        int64_t m = node_id(o, l, y);
        if (m >= 0 && L->solid[m]) {
          double cd = 0;
          for (int a = 0; a < 3; ++a) cd += o->c[i][a] * ob->dir[a];
          lo[i] += 2.0 * cd / ob->nsub;
        }
      }
    }
    double F[3], lFn[3] = {0, 0, 0}, lin[OMAXQ];
    node_force(o, l, n, F);
    ora_kbc_adj(o->D, L->beta, &g[(size_t)n * Q], F, lo, lin, lFn);
    for (int i = 0; i < Q; ++i) {
      L->lg[(size_t)n * Q + i] += lin[i];
      lo[i] = 0.0;
    }
    /* the node force is (uniform + field) / 2^l */
    double s = 1.0 / (double)(1 << l);
    for (int a = 0; a < 3; ++a) L->lF[3 * n + a] += lFn[a] * s;
  }
}

/* composite point value source: 1 = child node, 0 = parent node */
static int point_src(const ora_t *o, int lp, const int64_t Xin[3], int64_t *node) {
  int64_t X[3] = {Xin[0], Xin[1], Xin[2]};
  canon(o, lp, X);
  int64_t xc[3] = {2 * X[0], 2 * X[1], 2 * X[2]};
  if (canon(o, lp + 1, xc) && in_region(o, lp + 1, xc) && dist_at(o, lp + 1, xc) >= 2) {
    *node = node_id(o, lp + 1, xc);
    return 1;
  }
  *node = node_id(o, lp, X);
  return 0;
}

/* reverse of couple with snapshots gp (parent) and gc (child) of the inputs */
static void adj_couple(ora_t *o, int lp, const double *gp, const double *gc) {
  olevel *P = &o->lev[lp], *C = &o->lev[lp + 1];
  int Q = o->Q, D = o->D;
  static const double w4[4] = {-1.0 / 16.0, 9.0 / 16.0, 9.0 / 16.0, -1.0 / 16.0};
  double fac_pc = P->beta / (2.0 * C->beta), fac_cp = 2.0 * C->beta / P->beta;
  /* adjoints of the written values, then clear them */
  double *lwc = (double *)calloc((size_t)(C->nn ? C->nn : 1) * Q, sizeof(double));
  double *lwp = (double *)calloc((size_t)(P->nn ? P->nn : 1) * Q, sizeof(double));
  for (int64_t n = 0; n < C->nn; ++n)
    if (!C->solid[n] && C->pd[n] <= 1)
      for (int i = 0; i < Q; ++i) {
        lwc[(size_t)n * Q + i] = C->lg[(size_t)n * Q + i];
        C->lg[(size_t)n * Q + i] = 0.0;
      }
  for (int64_t n = 0; n < P->nn; ++n)
    if (P->ring[n])
      for (int i = 0; i < Q; ++i) {
        lwp[(size_t)n * Q + i] = P->lg[(size_t)n * Q + i];
        P->lg[(size_t)n * Q + i] = 0.0;
      }
  /* fine interface nodes: g = f^eq(rho~, u~) + n~, tensor interpolation of points */
  for (int64_t n = 0; n < C->nn; ++n) {
    if (C->solid[n] || C->pd[n] > 1) continue;
    const int64_t *x = &C->pos[3 * n];
    int npt[3] = {1, 1, 1};
    int64_t pts[3][4];
    double wts[3][4];
    for (int a = 0; a < 3; ++a) {
      if (a < D && (x[a] & 1)) {
        npt[a] = 4;
        for (int k = 0; k < 4; ++k) {
          pts[a][k] = (x[a] - 3 + 2 * k) / 2;
          wts[a][k] = w4[k];
        }
      } else {
        pts[a][0] = x[a] / 2;
        wts[a][0] = 1.0;
      }
    }
    /* forward values at the node */
    double rr = 0, uu[3] = {0, 0, 0};
    for (int kz = 0; kz < npt[2]; ++kz)
      for (int ky = 0; ky < npt[1]; ++ky)
        for (int kx = 0; kx < npt[0]; ++kx) {
          int64_t X[3] = {pts[0][kx], pts[1][ky], pts[2][kz]}, m;
          double w = wts[0][kx] * wts[1][ky] * wts[2][kz], r, u[3], fn[OMAXQ];
          int ch = point_src(o, lp, X, &m);
          node_macro(o, ch ? &gc[(size_t)m * Q] : &gp[(size_t)m * Q], &r, u, fn);
          rr += w * r;
          for (int a = 0; a < 3; ++a) uu[a] += w * u[a];
        }
    const double *lR = &lwc[(size_t)n * Q];
    double lr = 0, lu[3] = {0, 0, 0};
    feq_T(D, rr, uu, lR, &lr, lu);
    for (int kz = 0; kz < npt[2]; ++kz)
      for (int ky = 0; ky < npt[1]; ++ky)
        for (int kx = 0; kx < npt[0]; ++kx) {
          int64_t X[3] = {pts[0][kx], pts[1][ky], pts[2][kz]}, m;
          double w = wts[0][kx] * wts[1][ky] * wts[2][kz];
          int ch = point_src(o, lp, X, &m);
          double lrw = w * lr, luw[3] = {w * lu[0], w * lu[1], w * lu[2]}, lnw[OMAXQ];
          for (int i = 0; i < Q; ++i) lnw[i] = w * lR[i];
          if (ch) macro_T(o, &gc[(size_t)m * Q], 1.0, lrw, luw, lnw, &C->lg[(size_t)m * Q]);
          else macro_T(o, &gp[(size_t)m * Q], fac_pc, lrw, luw, lnw, &P->lg[(size_t)m * Q]);
        }
  }
  /* parent ring: g = f^eq + fac_cp (g_c - f^eq) with (rho, u) of the fine twin g_c */
  for (int64_t n = 0; n < P->nn; ++n) {
    if (!P->ring[n]) continue;
    int64_t xc[3] = {2 * P->pos[3 * n], 2 * P->pos[3 * n + 1], 2 * P->pos[3 * n + 2]};
    int64_t m = node_id(o, lp + 1, xc);
    const double *lw = &lwp[(size_t)n * Q];
    double lnn[OMAXQ], r = 0, u[3] = {0, 0, 0}, fn[OMAXQ], lr = 0, lu[3] = {0, 0, 0}, lfe[OMAXQ];
    /* value = feq + fac (g - feq) = fac g + (1 - fac) feq(rho(g), u(g)) */
    node_macro(o, &gc[(size_t)m * Q], &r, u, fn);
    for (int i = 0; i < Q; ++i) {
      C->lg[(size_t)m * Q + i] += fac_cp * lw[i];
      lfe[i] = (1.0 - fac_cp) * lw[i];
      lnn[i] = 0.0;
    }
    feq_T(D, r, u, lfe, &lr, lu);
    macro_T(o, &gc[(size_t)m * Q], 0.0, lr, lu, lnn, &C->lg[(size_t)m * Q]);
  }
  free(lwc);
  free(lwp);
}

/* Run n coarse steps forward from the current state, evaluating the objective, then
 * the reverse sweep.  Afterwards the state is the final forward state; the adjoint of
 * the initial state and the force-field gradient are available from
 * ora_adjoint_state / ora_adjoint_force. */
int ora_adjoint_run(ora_t *o, int n, int objective, int body_level, const double dir[3], double *J_out) {
  if (!o->finalized) return fail(o, -2, "adjoint before finalize");
  if (objective == 0 && (body_level < 0 || body_level >= o->L)) return fail(o, -1, "bad body level");
  int Q = o->Q;
  /* states s_0 .. s_n */
  double **states = (double **)calloc((size_t)(n + 1) * o->L, sizeof(double *));
  for (int l = 0; l < o->L; ++l) {
    olevel *L = &o->lev[l];
    free(L->lf);
    free(L->lg);
    free(L->lF);
    L->lf = (double *)calloc((size_t)(L->nn ? L->nn : 1) * Q, sizeof(double));
    L->lg = (double *)calloc((size_t)(L->nn ? L->nn : 1) * Q, sizeof(double));
    L->lF = (double *)calloc((size_t)(L->nn ? L->nn : 1) * 3, sizeof(double));
    states[l] = dup_arr(L->f, (size_t)L->nn * Q);
  }
  oadj_obj ob;
  ob.objective = objective;
  ob.body_level = body_level;
  for (int a = 0; a < 3; ++a) ob.dir[a] = dir ? dir[a] : 0.0;
  ob.nsub = objective == 0 ? (double)n * (double)(1 << body_level) : 1.0;
  int rc = 0;
  double J = 0;
  if (objective == 0) ora_drag(o, body_level, (double[3]){0, 0, 0}, NULL, 1);
  for (int k = 1; k <= n && !rc; ++k) {
    rc = ora_advance(o, 1);
    for (int l = 0; l < o->L; ++l) states[(size_t)k * o->L + l] = dup_arr(o->lev[l].f, (size_t)o->lev[l].nn * Q);
  }
  if (rc) goto done;
  if (objective == 0) {
    double F[3];
    int64_t st;
    ora_drag(o, body_level, F, &st, 1);
    J = (F[0] * ob.dir[0] + F[1] * ob.dir[1] + F[2] * ob.dir[2]) / ob.nsub;
  } else {
    /* J = 1/2 sum_l sum_x w rho |u|^2 with rho u = j - F/2 at the final state */
    for (int l = 0; l < o->L; ++l) {
      olevel *L = &o->lev[l];
      for (int64_t m = 0; m < L->nn; ++m) {
        if (L->w[m] == 0.0) continue;
        double r = 0, j[3] = {0, 0, 0}, F[3];
        for (int i = 0; i < Q; ++i) {
          r += L->f[(size_t)m * Q + i];
          for (int a = 0; a < 3; ++a) j[a] += o->c[i][a] * L->f[(size_t)m * Q + i];
        }
        node_force(o, l, m, F);
        double p[3] = {j[0] - 0.5 * F[0], j[1] - 0.5 * F[1], j[2] - 0.5 * F[2]};
        double p2 = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
        J += 0.5 * L->w[m] * p2 / r;
        for (int i = 0; i < Q; ++i) {
          double pc = p[0] * o->c[i][0] + p[1] * o->c[i][1] + p[2] * o->c[i][2];
          L->lf[(size_t)m * Q + i] += L->w[m] * (pc / r - 0.5 * p2 / (r * r));
        }
        double s = 1.0 / (double)(1 << l);
        for (int a = 0; a < 3; ++a) L->lF[3 * m + a] += -0.5 * L->w[m] * p[a] / r * s;
      }
    }
  }
  /* reverse sweep over coarse steps */
  for (int k = n; k >= 1 && !rc; --k) {
    for (int l = 0; l < o->L; ++l)
      memcpy(o->lev[l].f, states[(size_t)(k - 1) * o->L + l], sizeof(double) * (size_t)o->lev[l].nn * Q);
    o->taping = 1;
    tape_clear(o);
    rc = ora_advance(o, 1);
    o->taping = 0;
    if (rc) break;
    for (int t = o->ntape - 1; t >= 0; --t) {
      otape *tp = &o->tape[t];
      if (tp->op == 0) adj_stream(o, tp->level);
      else if (tp->op == 1) adj_collide(o, tp->level, tp->skip, tp->g0, &ob);
      else adj_couple(o, tp->level, tp->g0, tp->g1);
    }
    tape_clear(o);
  }
  /* leave the final forward state */
  for (int l = 0; l < o->L; ++l)
    memcpy(o->lev[l].f, states[(size_t)n * o->L + l], sizeof(double) * (size_t)o->lev[l].nn * Q);
  if (objective == 0) ora_drag(o, body_level, (double[3]){0, 0, 0}, NULL, 1);
done:
  for (size_t k = 0; k < (size_t)(n + 1) * o->L; ++k) free(states[k]);
  free(states);
  if (J_out) *J_out = J;
  return rc;
}

/* adjoint of the initial post-collision state, dense [Q][box] */
int ora_adjoint_state(const ora_t *o, int l, double *out) {
  if (!o->finalized || l < 0 || l >= o->L || !o->lev[l].lf) return -1;
  const olevel *L = &o->lev[l];
  int64_t tot = L->bn[0] * L->bn[1] * L->bn[2];
  for (int64_t k = 0; k < tot; ++k) {
    int32_t n = L->id[k];
    for (int i = 0; i < o->Q; ++i) out[i * tot + k] = (n < 0 || L->solid[n]) ? 0.0 : L->lf[(size_t)n * o->Q + i];
  }
  return 0;
}

/* gradient with respect to the per-node force-density field of a level (level-0
 * units), dense [D][box] */
int ora_adjoint_force(const ora_t *o, int l, double *out) {
  if (!o->finalized || l < 0 || l >= o->L || !o->lev[l].lF) return -1;
  const olevel *L = &o->lev[l];
  int64_t tot = L->bn[0] * L->bn[1] * L->bn[2];
  for (int64_t k = 0; k < tot; ++k) {
    int32_t n = L->id[k];
    for (int a = 0; a < o->D; ++a) out[a * tot + k] = (n < 0 || L->solid[n]) ? 0.0 : L->lF[3 * n + a];
  }
  return 0;
}

/* gradient with respect to the initial velocity field, through
 * f_i = f^eq_i(rho0, u0)(1 + noise_i); lam = adjoint of the initial state [Q][box] */
int ora_init_adjoint_u(int D, int64_t tot, const double *rho, const double *u, const double *noise,
                       const double *lam, double *out) {
  int Q = D == 2 ? 9 : 27;
  for (int64_t k = 0; k < tot; ++k) {
    double uu[3] = {0, 0, 0}, lr = 0, lu[3] = {0, 0, 0}, lf[OMAXQ];
    for (int a = 0; a < D; ++a) uu[a] = u[a * tot + k];
    for (int i = 0; i < Q; ++i) lf[i] = lam[i * tot + k] * (noise ? 1.0 + noise[i * tot + k] : 1.0);
    feq_T(D, rho[k], uu, lf, &lr, lu);
    for (int a = 0; a < D; ++a) out[a * tot + k] = lu[a];
  }
  return 0;
}
