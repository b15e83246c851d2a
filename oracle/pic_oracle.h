/*
 * pic_oracle.h — plain FP64 CPU oracle of the particle hot path of the
 * extended particle-in-cell methods for sheared, expanding or escaping plasma
 * (Bacchini et al., arXiv 2602.15939).
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  It shares no code with the
 * HIP path and the HIP path never calls it.
 *
 * Code units: c = 1, cell size dx = 1, Gaussian units with an explicit 4*pi.
 * Grid: Yee lattice.  Node (i,j,k) sits at integer coordinates; component
 * offsets in cells:
 *   Ex (1/2,0,0)  Ey (0,1/2,0)  Ez (0,0,1/2)     J as E
 *   Bx (0,1/2,1/2) By (1/2,0,1/2) Bz (1/2,1/2,0)
 * A field component array holds n[0]*n[1]*n[2] values, x fastest.
 * In 2D (dim = 2) n[2] = 1 and every z derivative is zero.
 * Particle positions are FP64 global coordinates X in [0, n[d]).
 * For the shearing box the radial coordinate of the paper is x = X - n[0]/2.
 */
#ifndef PIC_ORACLE_H
#define PIC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORA_PLAIN = 0, ORA_SHEAR = 1, ORA_EXPAND = 2, ORA_LEAKY = 3, ORA_SHEAR_EXPAND = 4 };
enum { ORA_LEAKY_DISPLACEMENT = 0, ORA_LEAKY_PROBABILISTIC = 1 };
enum { ORA_EXPAND_PRINTED = 0, ORA_EXPAND_EXACT = 1 };

/* Extended current grid: x gets ORA_JG guard columns on each side, y and z wrap. */
#define ORA_JG 3

typedef struct ora_box {
    int dim;            /* 2 or 3 */
    int n[3];           /* cells per axis, n[2] = 1 in 2D */
    double dt;          /* time step */
    int frame;          /* ORA_PLAIN / ORA_SHEAR / ORA_EXPAND / ORA_LEAKY / ORA_SHEAR_EXPAND */
    /* shearing box (section 2): v_s = -s*Omega0*x e_y */
    double shear_s, omega0;
    /* expanding box (section 3): l_d(t) = 1 + adot*t on the axes set in axis_mask; the
       combined frame takes masks that scale x and y together (0, z, xy, xyz) */
    double adot;
    int axis_mask;
    int expand_push;    /* ORA_EXPAND_PRINTED (the method) or ORA_EXPAND_EXACT (3x3 solve) */
    /* leaky box (section 4) */
    int leaky_mode;     /* ORA_LEAKY_DISPLACEMENT or ORA_LEAKY_PROBABILISTIC */
    double l_esc;       /* displacement mode: escape distance */
    int use_3vec;       /* displacement mode: 1 = test all three components */
    double t_esc;       /* probabilistic mode: mean escape time */
    double gamma_thr;   /* probabilistic mode: Lorentz factor threshold */
    int reinject;       /* unused by the oracle (no reinjection in probabilistic mode) */
    uint64_t seed;      /* Philox key */
    uint32_t box_id;    /* fourth Philox counter word */
    const double* mj_table; /* displacement mode: inverse CDF of |u|, mj_bins+mj_tail values */
    int mj_bins, mj_tail;
    /* Maxwell (shearing box): fixed-point iterations and tolerance (0 = fixed count) */
    int maxwell_iters;
    double maxwell_tol;
    int64_t step;       /* n of the step about to be taken; t^n = n*dt */
    int last_iters;     /* output: iterations used by the last shearing-box Maxwell solve */
    int64_t n_superluminal; /* output, accumulated: shearing-box pushes whose effective
                               velocity u'/gamma' + v_s (v_s at the midpoint x) exceeds c */
    int escape;         /* the leaky box's escape rule in the shearing or expanding frame too
                           (implied by ORA_LEAKY), on the displacement the deposit uses */
} ora_box;

typedef struct ora_species {
    int64_t n;
    double q_over_m;    /* charge-to-mass ratio (sign included) */
    double q;           /* macro-particle charge (sign included) */
    double *x, *y, *z;  /* positions (z unused in 2D) */
    double *ux, *uy, *uz;
    double *drx, *dry, *drz; /* leaky displacement (may be NULL otherwise) */
    uint32_t* id;
    uint8_t* alive;     /* 1 = live; probabilistic escape clears it */
} ora_species;

typedef struct ora_fields {
    double *E[3], *B[3], *J[3];
} ora_fields;

/* ---- helpers exposed for the tests ---- */
double ora_shear_offset(const ora_box* b, double t);   /* Delta y_s(t) reduced mod n[1] */
double ora_scale(const ora_box* b, int axis, double t); /* l_axis(t) */

void ora_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void ora_philox_many(int64_t n, const uint32_t* ctr4, const uint32_t* key2, uint32_t* out4);

void ora_mj_table(double theta, int nbins, int ntail, double* table);
void ora_mj_sample(const double* table, int nbins, int ntail, const uint32_t w[4], double u[3]);

/* stable counting sort: perm lists the indices with key < nkeys in key order;
   offsets has nkeys+2 entries, the last bin (key == nkeys) is the dead bin. */
void ora_stable_sort(int64_t n, const int32_t* keys, int32_t nkeys, int64_t* perm,
                     int64_t* offsets);

/* gather: fields at n positions (global coordinates), shear offset dys for the x guards */
void ora_gather(const ora_box* b, const ora_fields* f, double dys, int64_t n,
                const double* x, const double* y, const double* z, double* Eo, double* Bo);

/* per-particle pushers; E,B are 3*n interleaved at the particles, u is 3*n interleaved.
   xr = radial coordinate x (shear only).  Returns u^{n+1/2} in place. */
void ora_push_boris(int64_t n, double qm, double dt, const double* E, const double* B,
                    double* u);
void ora_push_shear(int64_t n, double qm, double dt, double s, double omega0,
                    const double* xr, const double* E, const double* B, double* u,
                    double* gbar_out);
void ora_push_expand(int64_t n, double qm, double dt, const double lam[3], int exact,
                     const double* E, const double* B, double* u);
double ora_shear_gamma_bar(double A, double K);
/* shearing and expanding frame combined (reading of the extension named in Sec. 5): the
   rank-1 S and Coriolis tau~ of eq. OAu_disc with the diagonal Lambda of eq. EBu_disc;
   exact != 0 solves the 3x3 system instead of the printed-style closed form */
void ora_push_shear_expand(int64_t n, double qm, double dt, double s, double omega0,
                           const double lam[3], int exact, const double* xr, const double* E,
                           const double* B, double* u, double* gbar_out);

/* Esirkepov deposit of n particles moving x0 -> x1 (global coordinates; x1 not wrapped),
   into the extended current grid Jext (3 components, (n0+2*ORA_JG)*n1*n2 each).
   dz = z displacement (2D J_z). */
void ora_deposit(const ora_box* b, int64_t n, double q, const double* x0, const double* y0,
                 const double* z0, const double* x1, const double* y1, const double* z1,
                 const double* dz, double* Jext);
/* fold the extended grid into J (n0*n1*n2), with the shear advection and shearing-periodic
   fold for ORA_SHEAR; t_half = time of the current */
void ora_finalize_current(const ora_box* b, const double* Jext, double* J, double t_half);

/* one Maxwell step of the box frame; uses b->step for the time levels */
void ora_maxwell(ora_box* b, ora_fields* f);
/* right-hand side of the shearing-box field equations at the fields (E,B) whose x guards
   use shear offset dys; out = 6 arrays (dB/dt then dE'/dt) */
void ora_ksb_rhs(const ora_box* b, double* const E[3], double* const B[3], double dys,
                 double* const J[3], double* const out[6]);
/* the same with the expanding-frame factors of the combined frame: the curls act on d_c F_c,
   the transport term v dE'y/dz of dE'z/dt carries kz */
void ora_ksb_rhs_f(const ora_box* b, double* const E[3], double* const B[3], double dys,
                   double* const J[3], const double d[3], double kz, double* const out[6]);

/* charge density at nodes of n particles (CIC) into rho (n0*n1*n2), added */
void ora_charge(const ora_box* b, int64_t n, double q, const double* x, const double* y,
                const double* z, double* rho);

/* one full step of the box frame for all species (step order of sections 2.2, 3.2, 4.1) */
int ora_step(ora_box* b, ora_fields* f, ora_species* sp, int nsp, int nthreads);
/* the particle part of a step only (gather, push, move, leaky escape): no deposit, no
   Maxwell, b->step unchanged */
int ora_particles_only(ora_box* b, const ora_fields* f, ora_species* sp, int nsp);

/* FP64 diagnostics: out[0..2] = sum E_c^2/8pi, out[3..5] = sum B_c^2/8pi,
   out[6] = kinetic energy sum m(gamma-1), out[7..9] = momentum sum m u, out[10] = live count */
void ora_energies(const ora_box* b, const ora_fields* f, const ora_species* sp, int nsp,
                  double* out);

/* FP32 integer-semantics layer: the in-cell offset renormalisation used by the FP32 path
   (int32 cell + FP32 offset).  Applies off + delta in FP32 and renormalises to [0,1). */
void ora_f32_normalize(int64_t n, const int32_t* cell, const float* off, const float* delta,
                       int32_t* cell_out, float* off_out);
/* FP32 integer layer of the position update: cell (linear) + offsets (dim x n) moved by the
   FP32 deposit displacement disp (3 x n) with the frame's shear move and boundaries at
   t^{n+1} = (b->step + 1) dt; err[p] = 1 where the displacement breaks the step bounds. */
void ora_f32_move(const ora_box* b, int64_t n, const int32_t* cell, const float* off,
                  const float* disp, int32_t* cell_out, float* off_out, uint8_t* err);
/* tile key of the cell (i,j,k) for tile shape t[3], dead particles (i < 0) -> n_tiles */
void ora_tile_keys(const ora_box* b, const int t[3], int64_t n, const int32_t* ci,
                   const int32_t* cj, const int32_t* ck, int32_t* keys);

#ifdef __cplusplus
}
#endif
#endif
