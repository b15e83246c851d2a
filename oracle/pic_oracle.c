/*
 * pic_oracle.c — plain FP64 CPU oracle of the particle hot path of the extended
 * particle-in-cell methods of Bacchini et al. (arXiv 2602.15939): field gather,
 * the generalised Boris-like pushers of the shearing box (Sec. 2.2) and the
 * expanding box (Sec. 3.2), the leaky-box escape (Sec. 4.1), charge-conserving
 * current deposition, the current finalisation with the shear transport of J'
 * (Sec. 2.2) and the shearing-periodic boundaries (Sec. 2.1), and the Maxwell
 * solvers of each frame.
 *
 * TEST INFRASTRUCTURE: loaded only by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark.  It shares no code with the HIP path.
 *
 * Everything is written in the plainest form of the paper's equations, in FP64,
 * with no blocking, fusion or reordering.  Readings of points the paper leaves
 * open are marked "reading:".
 */
#include "pic_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORA_PI 3.14159265358979323846

/* ------------------------------------------------------------------ */
/* indexing                                                            */
/* ------------------------------------------------------------------ */

static inline int wrapi(int i, int n)
{
    i %= n;
    return i < 0 ? i + n : i;
}

static inline int64_t cidx(const ora_box* b, int i, int j, int k)
{
    return (int64_t)i + (int64_t)b->n[0] * ((int64_t)j + (int64_t)b->n[1] * k);
}

static inline int64_t ncells(const ora_box* b)
{
    return (int64_t)b->n[0] * b->n[1] * b->n[2];
}

/* Yee offsets (in cells) of E (and J) and B components */
static const double STAG_E[3][3] = {{0.5, 0, 0}, {0, 0.5, 0}, {0, 0, 0.5}};
static const double STAG_B[3][3] = {{0, 0.5, 0.5}, {0.5, 0, 0.5}, {0.5, 0.5, 0}};

/* ------------------------------------------------------------------ */
/* frame scalars                                                       */
/* ------------------------------------------------------------------ */

/* Sec. 2.1: Delta y_s = s Omega0 (x_o - x_i) t, reduced modulo the box length in y */
/* frames with the shearing-box geometry (Sec. 2) and with the expanding-box scale factors
   (Sec. 3); the combined frame has both */
static inline int sheared(const ora_box* b)
{
    return b->frame == ORA_SHEAR || b->frame == ORA_SHEAR_EXPAND;
}
static inline int expanding(const ora_box* b)
{
    return b->frame == ORA_EXPAND || b->frame == ORA_SHEAR_EXPAND;
}

/* Sec. 2.1: Delta y_s = s Omega0 (x_o - x_i) t.  In the combined frame x and y scale together
   (reading), so the shear flow in the expanding coordinates, -s Omega0 (l_x/l_y) x', and with
   it Delta y_s, keep their form. */
double ora_shear_offset(const ora_box* b, double t)
{
    if (!sheared(b)) return 0.0;
    double ny = (double)b->n[1];
    double d = b->shear_s * b->omega0 * (double)b->n[0] * t;
    d = fmod(d, ny);
    if (d < 0) d += ny;
    if (d >= ny) d = 0.0;
    return d;
}

/* Sec. 3.1: L = diag(l_1, l_2, l_3); reading: l_d = a(t) = 1 + adot t on the expanding axes */
double ora_scale(const ora_box* b, int axis, double t)
{
    if (!expanding(b)) return 1.0;
    if (!((b->axis_mask >> axis) & 1)) return 1.0;
    return 1.0 + b->adot * t;
}

static double scale_rate(const ora_box* b, int axis)
{
    if (!expanding(b)) return 0.0;
    if (!((b->axis_mask >> axis) & 1)) return 0.0;
    return b->adot;
}

/* ------------------------------------------------------------------ */
/* field access with the boundary conditions                          */
/* ------------------------------------------------------------------ */

/* Value of component array F at lattice index (i,j,k); y and z are periodic.  In x the
   shearing box uses the shearing-periodic condition of Sec. 2.1, F(x_i, y) = F(x_o, y - dys):
   a lattice point beyond x_o maps to (x - Lx, y + dys), one below x_i to (x + Lx, y - dys).
   reading: a fractional dys is applied by linear interpolation along y. */
static double fget(const ora_box* b, const double* F, int i, int j, int k, double dys)
{
    const int nx = b->n[0], ny = b->n[1], nz = b->n[2];
    k = wrapi(k, nz);
    if (i >= 0 && i < nx) return F[cidx(b, i, wrapi(j, ny), k)];
    if (!sheared(b)) return F[cidx(b, wrapi(i, nx), wrapi(j, ny), k)];
    double sh;
    int ii;
    if (i >= nx) {
        sh = dys;
        ii = i - nx;
    } else {
        sh = -dys;
        ii = i + nx;
    }
    double fl = floor(sh);
    int js = (int)fl;
    double w = sh - fl;
    double a = F[cidx(b, ii, wrapi(j + js, ny), k)];
    double c = F[cidx(b, ii, wrapi(j + js + 1, ny), k)];
    return (1.0 - w) * a + w * c;
}

/* A field seen through a weighted pair of arrays, each with its own shear offset; used for
   the implicit-midpoint average (F^n + F^k)/2 whose two members sit at different times. */
typedef struct {
    const double* a;
    const double* c;
    double dys_a, dys_c;
    double wa, wc;
} facc;

static inline double fv(const ora_box* b, const facc* f, int i, int j, int k)
{
    double v = f->wa * fget(b, f->a, i, j, k, f->dys_a);
    if (f->wc != 0.0) v += f->wc * fget(b, f->c, i, j, k, f->dys_c);
    return v;
}

/* ------------------------------------------------------------------ */
/* gather (Sec. 1: fields interpolated from the grid to the particles) */
/* ------------------------------------------------------------------ */

/* reading: each component is interpolated with linear (CIC) weights on its own staggered
   lattice */
static double interp(const ora_box* b, const double* F, const double st[3], double X, double Y,
                     double Z, double dys)
{
    const int nd = b->dim;
    double pos[3] = {X - st[0], Y - st[1], Z - st[2]};
    int base[3] = {0, 0, 0};
    double w[3] = {0, 0, 0};
    for (int d = 0; d < nd; d++) {
        double fl = floor(pos[d]);
        base[d] = (int)fl;
        w[d] = pos[d] - fl;
    }
    double acc = 0.0;
    for (int c = 0; c < (1 << nd); c++) {
        int ii[3] = {base[0], base[1], base[2]};
        double wt = 1.0;
        for (int d = 0; d < nd; d++) {
            int bit = (c >> d) & 1;
            ii[d] += bit;
            wt *= bit ? w[d] : 1.0 - w[d];
        }
        acc += wt * fget(b, F, ii[0], ii[1], ii[2], dys);
    }
    return acc;
}

void ora_gather(const ora_box* b, const ora_fields* f, double dys, int64_t n, const double* x,
                const double* y, const double* z, double* Eo, double* Bo)
{
    for (int64_t p = 0; p < n; p++) {
        double Z = (b->dim == 3 && z) ? z[p] : 0.0;
        for (int c = 0; c < 3; c++) {
            Eo[3 * p + c] = interp(b, f->E[c], STAG_E[c], x[p], y[p], Z, dys);
            Bo[3 * p + c] = interp(b, f->B[c], STAG_B[c], x[p], y[p], Z, dys);
        }
    }
}

/* ------------------------------------------------------------------ */
/* vector helpers                                                      */
/* ------------------------------------------------------------------ */

static inline void cross(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static inline double dot(const double a[3], const double b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* Boris operator of Sec. 2.2: B(v) = v + 2 v x t/(1+t^2) + 2 (v x t) x t/(1+t^2) */
static void op_boris(const double v[3], const double t[3], double out[3])
{
    double vt[3], vtt[3];
    cross(v, t, vt);
    cross(vt, t, vtt);
    double den = 1.0 + dot(t, t);
    for (int c = 0; c < 3; c++) out[c] = v[c] + 2.0 * vt[c] / den + 2.0 * vtt[c] / den;
}

/* half-Boris rotation of Sec. 2.2: R(v) = v + v x t/(1+t^2) + (v x t) x t/(1+t^2) */
static void op_half(const double v[3], const double t[3], double out[3])
{
    double vt[3], vtt[3];
    cross(v, t, vt);
    cross(vt, t, vtt);
    double den = 1.0 + dot(t, t);
    for (int c = 0; c < 3; c++) out[c] = v[c] + vt[c] / den + vtt[c] / den;
}

/* ------------------------------------------------------------------ */
/* pushers                                                             */
/* ------------------------------------------------------------------ */

/* Standard Boris push (the alpha = 0 limit of Sec. 2.2 and the Lambda = 0 limit of Sec. 3.2) */
void ora_push_boris(int64_t n, double qm, double dt, const double* E, const double* B, double* u)
{
    for (int64_t p = 0; p < n; p++) {
        double eps[3], um[3], tau[3], up[3];
        for (int c = 0; c < 3; c++) {
            eps[c] = qm * dt * E[3 * p + c] / 2.0;
            um[c] = u[3 * p + c] + eps[c];
        }
        double gbar = sqrt(1.0 + dot(um, um));
        for (int c = 0; c < 3; c++) tau[c] = qm * dt * B[3 * p + c] / (2.0 * gbar);
        op_boris(um, tau, up);
        for (int c = 0; c < 3; c++) u[3 * p + c] = up[c] + eps[c];
    }
}

/* gamma-bar of the shearing-box push (Sec. 2.2): the real root >= 1 of
       g^2 = 1 + A + K/g,   i.e.  g^3 - (1+A) g - K = 0,
   with A = (u^-)^2 + 2 alpha1 u^-_x u^-_y and K = 2 alpha2 (u^- . eps) u^-_y (c = 1).
   reading: the largest real root.  Newton from a point above it converges monotonically
   because the cubic is convex and increasing there. */
double ora_shear_gamma_bar(double A, double K)
{
    double g = sqrt(1.0 + A) + fabs(K) + 1.0;
    for (int it = 0; it < 200; it++) {
        double f = g * g * g - (1.0 + A) * g - K;
        double fp = 3.0 * g * g - (1.0 + A);
        double gn = g - f / fp;
        if (!(gn < g)) break; /* monotone from above: stop when no further decrease */
        g = gn;
    }
    return g;
}

/* Shearing-box push, eq. (OAu_disc) of Sec. 2.2 solved by the printed closed form
       u+ = B(u-) + R(S u-) + R(S(B(u-) + R(S u-))) / (1 - g),  g = S_2 . R(e_y)
   with eps = q dt E'/2m, eps~ = eps/(c gbar), tau = q dt B/(2mc), tau~ = tau/gbar + dt Omega0,
   alpha1 = s Omega0 dt/2, alpha2 = s Omega0 x^n / c, and u'^{n+1/2} = u+ + eps. */
void ora_push_shear(int64_t n, double qm, double dt, double s, double omega0, const double* xr,
                    const double* E, const double* B, double* u, double* gbar_out)
{
    const double a1 = s * omega0 * dt / 2.0;
    for (int64_t p = 0; p < n; p++) {
        const double a2 = s * omega0 * xr[p];
        double eps[3], um[3];
        for (int c = 0; c < 3; c++) {
            eps[c] = qm * dt * E[3 * p + c] / 2.0;
            um[c] = u[3 * p + c] + eps[c];
        }
        double A = dot(um, um) + 2.0 * a1 * um[0] * um[1];
        double K = 2.0 * a2 * dot(um, eps) * um[1];
        double gbar = ora_shear_gamma_bar(A, K);
        if (gbar_out) gbar_out[p] = gbar;
        double tt[3], et[3];
        for (int c = 0; c < 3; c++) {
            tt[c] = qm * dt * B[3 * p + c] / 2.0 / gbar;
            et[c] = eps[c] / gbar;
        }
        tt[2] += dt * omega0; /* Omega0 = (0, 0, Omega0) */
        /* S: rank-1, only row y is non-zero: (alpha1 + alpha2 eps~_x, alpha2 eps~_y, alpha2 eps~_z) */
        double s2[3] = {a1 + a2 * et[0], a2 * et[1], a2 * et[2]};
        double Bu[3], Su[3] = {0, 0, 0}, RSu[3], w[3], Sw[3] = {0, 0, 0}, RSw[3];
        op_boris(um, tt, Bu);
        Su[1] = dot(s2, um);
        op_half(Su, tt, RSu);
        for (int c = 0; c < 3; c++) w[c] = Bu[c] + RSu[c];
        Sw[1] = dot(s2, w);
        op_half(Sw, tt, RSw);
        double ey[3] = {0, 1, 0}, Rey[3];
        op_half(ey, tt, Rey);
        double g = dot(s2, Rey);
        for (int c = 0; c < 3; c++) u[3 * p + c] = w[c] + RSw[c] / (1.0 - g) + eps[c];
    }
}

/* Expanding-box push, eq. (EBu_disc) of Sec. 3.2 with the printed modified Boris operator
     B^(L)(v) = L~ v + ((1+L~) v x tau~)/(1+tau~^2) + (((1+L~) v x tau~) x tau~)/(1+tau~^2),
   tau~_i = tau_i/(1-Lambda_ii), L~_ii = (1+Lambda_ii)/(1-Lambda_ii),
   gbar = sqrt(1 + ((1+Lambda) u-)^2/c^2), tau = q dt B/(2 gbar m c).
   lam holds the diagonal of Lambda = -(dt/2) L^-1 dL/dt.  exact != 0 solves
   (1 - Lambda - T) u+ = (1 + Lambda + T) u- with a 3x3 Gaussian elimination instead
   (ablation only). */
void ora_push_expand(int64_t n, double qm, double dt, const double lam[3], int exact,
                     const double* E, const double* B, double* u)
{
    for (int64_t p = 0; p < n; p++) {
        double eps[3], um[3], lu[3];
        for (int c = 0; c < 3; c++) {
            eps[c] = qm * dt * E[3 * p + c] / 2.0;
            um[c] = u[3 * p + c] + eps[c];
            lu[c] = (1.0 + lam[c]) * um[c];
        }
        double gbar = sqrt(1.0 + dot(lu, lu));
        double tau[3];
        for (int c = 0; c < 3; c++) tau[c] = qm * dt * B[3 * p + c] / (2.0 * gbar);
        double up[3];
        if (!exact) {
            double tt[3], Lt[3], w[3], wt[3], wtt[3];
            for (int c = 0; c < 3; c++) {
                tt[c] = tau[c] / (1.0 - lam[c]);
                Lt[c] = (1.0 + lam[c]) / (1.0 - lam[c]);
                w[c] = (1.0 + Lt[c]) * um[c];
            }
            cross(w, tt, wt);
            cross(wt, tt, wtt);
            double den = 1.0 + dot(tt, tt);
            for (int c = 0; c < 3; c++) up[c] = Lt[c] * um[c] + wt[c] / den + wtt[c] / den;
        } else {
            /* M u+ = r with M = diag(1-lam) - [tau x], r = (1+lam) u- + u- x tau,
               where [tau x] v = v x tau */
            double M[3][4];
            double ut[3];
            cross(um, tau, ut);
            for (int r = 0; r < 3; r++)
                for (int c = 0; c < 3; c++) M[r][c] = 0.0;
            for (int c = 0; c < 3; c++) M[c][c] = 1.0 - lam[c];
            /* v x tau = (v1 t2 - v2 t1, v2 t0 - v0 t2, v0 t1 - v1 t0): subtract its matrix */
            M[0][1] -= tau[2];
            M[0][2] += tau[1];
            M[1][0] += tau[2];
            M[1][2] -= tau[0];
            M[2][0] -= tau[1];
            M[2][1] += tau[0];
            for (int c = 0; c < 3; c++) M[c][3] = (1.0 + lam[c]) * um[c] + ut[c];
            for (int piv = 0; piv < 3; piv++) {
                int best = piv;
                for (int r = piv + 1; r < 3; r++)
                    if (fabs(M[r][piv]) > fabs(M[best][piv])) best = r;
                for (int c = 0; c < 4; c++) {
                    double tmp = M[piv][c];
                    M[piv][c] = M[best][c];
                    M[best][c] = tmp;
                }
                for (int r = 0; r < 3; r++) {
                    if (r == piv) continue;
                    double f = M[r][piv] / M[piv][piv];
                    for (int c = 0; c < 4; c++) M[r][c] -= f * M[piv][c];
                }
            }
            for (int c = 0; c < 3; c++) up[c] = M[c][3] / M[c][c];
        }
        for (int c = 0; c < 3; c++) u[3 * p + c] = up[c] + eps[c];
    }
}

/* 3x3 linear solve by Gaussian elimination with partial pivoting (augmented rows) */
static void solve3(double M[3][4], double x[3])
{
    for (int piv = 0; piv < 3; piv++) {
        int best = piv;
        for (int r = piv + 1; r < 3; r++)
            if (fabs(M[r][piv]) > fabs(M[best][piv])) best = r;
        for (int c = 0; c < 4; c++) {
            double tmp = M[piv][c];
            M[piv][c] = M[best][c];
            M[best][c] = tmp;
        }
        for (int r = 0; r < 3; r++) {
            if (r == piv) continue;
            double f = M[r][piv] / M[piv][piv];
            for (int c = 0; c < 4; c++) M[r][c] -= f * M[piv][c];
        }
    }
    for (int c = 0; c < 3; c++) x[c] = M[c][3] / M[c][c];
}

/* Combined shearing and expanding frame (the extension the conclusion, Sec. 5, names).
   reading: the discrete momentum equation adds the diagonal Lambda of eq. EBu_disc (Sec. 3.2)
   to eq. OAu_disc (Sec. 2.2),
       (1 - Lambda) u+ - u+ x tau~ - S u+ = (1 + Lambda) u- + u- x tau~ + S u-,
   with eps, eps~, tau~ = tau/gbar + dt Omega0, alpha1, alpha2 and the rank-1 S (only row y:
   s2 = (alpha1 + alpha2 eps~_x, alpha2 eps~_y, alpha2 eps~_z)) of Sec. 2.2 and
   Lambda = -(dt/2) L^-1 dL/dt of Sec. 3.2.  gbar takes both Boris-like definitions: the
   largest real root of gbar^2 = 1 + ((1+Lambda)u-)^2 + 2 alpha1 u-_x u-_y
   + 2 alpha2 (u-.eps) u-_y / gbar.  Closed form: A u = (1 - Lambda) u - u x tau~ is inverted
   as the expanding push does, A^-1 r = R_t((1 - Lambda)^-1 r) with t = (1 - Lambda)^-1 tau~
   (R the half rotation of Sec. 2.2), so that A^-1((1 + Lambda) v + v x tau~) is the printed
   modified Boris operator B^(Lambda)(v) of Sec. 3.2; the rank-1 S is added by the
   Sherman-Morrison formula, as the shearing push adds it to R:
       w = B^(Lambda)(u-) + (s2 . u-) A^-1 e_y,   g = s2 . A^-1 e_y,
       u+ = w + (s2 . w) A^-1 e_y / (1 - g),   u'^{n+1/2} = u+ + eps.
   Lambda = 0 gives the shearing push of Sec. 2.2, S = 0 with Omega0 = 0 the expanding push of
   Sec. 3.2.  exact != 0 solves the 3x3 system directly. */
void ora_push_shear_expand(int64_t n, double qm, double dt, double s, double omega0,
                           const double lam[3], int exact, const double* xr, const double* E,
                           const double* B, double* u, double* gbar_out)
{
    const double a1 = s * omega0 * dt / 2.0;
    for (int64_t p = 0; p < n; p++) {
        const double a2 = s * omega0 * xr[p];
        double eps[3], um[3], lu[3];
        for (int c = 0; c < 3; c++) {
            eps[c] = qm * dt * E[3 * p + c] / 2.0;
            um[c] = u[3 * p + c] + eps[c];
            lu[c] = (1.0 + lam[c]) * um[c];
        }
        const double A = dot(lu, lu) + 2.0 * a1 * um[0] * um[1];
        const double K = 2.0 * a2 * dot(um, eps) * um[1];
        const double gbar = ora_shear_gamma_bar(A, K);
        if (gbar_out) gbar_out[p] = gbar;
        double tt[3], et[3];
        for (int c = 0; c < 3; c++) {
            tt[c] = qm * dt * B[3 * p + c] / 2.0 / gbar;
            et[c] = eps[c] / gbar;
        }
        tt[2] += dt * omega0;
        const double s2[3] = {a1 + a2 * et[0], a2 * et[1], a2 * et[2]};
        double up[3];
        if (!exact) {
            double t[3], Lt[3], v[3], vt[3], vtt[3], Bu[3];
            for (int c = 0; c < 3; c++) {
                t[c] = tt[c] / (1.0 - lam[c]);
                Lt[c] = (1.0 + lam[c]) / (1.0 - lam[c]);
                v[c] = (1.0 + Lt[c]) * um[c];
            }
            cross(v, t, vt);
            cross(vt, t, vtt);
            const double den = 1.0 + dot(t, t);
            for (int c = 0; c < 3; c++) Bu[c] = Lt[c] * um[c] + vt[c] / den + vtt[c] / den;
            /* A^-1 e_y = R_t((1 - Lambda)^-1 e_y) */
            double ey[3] = {0.0, 1.0 / (1.0 - lam[1]), 0.0}, Ae[3];
            op_half(ey, t, Ae);
            const double g = dot(s2, Ae);
            const double su = dot(s2, um);
            double w[3];
            for (int c = 0; c < 3; c++) w[c] = Bu[c] + su * Ae[c];
            const double sw = dot(s2, w);
            for (int c = 0; c < 3; c++) up[c] = w[c] + sw * Ae[c] / (1.0 - g);
        } else {
            /* M u+ = r, M = diag(1 - lam) - [x tau~] - e_y s2^T, r = (1 + lam) u- + u- x tau~
               + e_y (s2 . u-), with [x t] v = v x t */
            double M[3][4], ut[3];
            cross(um, tt, ut);
            for (int r = 0; r < 3; r++)
                for (int c = 0; c < 3; c++) M[r][c] = 0.0;
            for (int c = 0; c < 3; c++) M[c][c] = 1.0 - lam[c];
            M[0][1] -= tt[2];
            M[0][2] += tt[1];
            M[1][0] += tt[2];
            M[1][2] -= tt[0];
            M[2][0] -= tt[1];
            M[2][1] += tt[0];
            for (int c = 0; c < 3; c++) M[1][c] -= s2[c];
            for (int c = 0; c < 3; c++) M[c][3] = (1.0 + lam[c]) * um[c] + ut[c];
            M[1][3] += dot(s2, um);
            solve3(M, up);
        }
        for (int c = 0; c < 3; c++) u[3 * p + c] = up[c] + eps[c];
    }
}

/* ------------------------------------------------------------------ */
/* Esirkepov charge-conserving deposit (CIC shape)                     */
/* ------------------------------------------------------------------ */

static inline double cic(double r)
{
    r = fabs(r);
    return r < 1.0 ? 1.0 - r : 0.0;
}

static inline int64_t jext_cells(const ora_box* b)
{
    return (int64_t)(b->n[0] + 2 * ORA_JG) * b->n[1] * b->n[2];
}

static inline double* jext_at(const ora_box* b, double* J, int c, int i, int j, int k)
{
    const int nxe = b->n[0] + 2 * ORA_JG;
    int64_t off = (int64_t)(i + ORA_JG) +
                  (int64_t)nxe * ((int64_t)wrapi(j, b->n[1]) + (int64_t)b->n[1] * wrapi(k, b->n[2]));
    return &J[c * jext_cells(b) + off];
}

#define SW 5 /* stencil width: nodes nearest-2 .. nearest+2 covers moves below 1.5 cells */

/* Esirkepov (2001) decomposition of the change of the CIC density S1 - S0 into the three
   current components, with W^x = DS_x (S0_y S0_z + DS_y S0_z/2 + S0_y DS_z/2 + DS_y DS_z/3)
   (cyclic) and J_x obtained by the running sum along x of -q W^x / dt.  In 2D,
   W^x = DS_x (S0_y + DS_y/2), W^y = DS_y (S0_x + DS_x/2) and
   J_z = q (dz/dt) (S0_x S0_y + DS_x S0_y/2 + S0_x DS_y/2 + DS_x DS_y/3). */
static void deposit_one(const ora_box* b, double q, const double X0[3], const double X1[3],
                        double dz, double* Jext)
{
    const int nd = b->dim;
    const double dt = b->dt;
    int nn[3] = {0, 0, 0};
    double S0[3][SW], S1[3][SW], DS[3][SW];
    for (int d = 0; d < 3; d++) {
        for (int a = 0; a < SW; a++) {
            S0[d][a] = S1[d][a] = DS[d][a] = 0.0;
        }
    }
    for (int d = 0; d < nd; d++) {
        nn[d] = (int)floor(X0[d] + 0.5);
        for (int a = 0; a < SW; a++) {
            double node = (double)(nn[d] + a - SW / 2);
            S0[d][a] = cic(node - X0[d]);
            S1[d][a] = cic(node - X1[d]);
            DS[d][a] = S1[d][a] - S0[d][a];
        }
    }
    if (nd == 3) {
        for (int bb = 0; bb < SW; bb++)
            for (int cc = 0; cc < SW; cc++) {
                double acc = 0.0;
                for (int a = 0; a < SW - 1; a++) {
                    double wx = DS[0][a] * (S0[1][bb] * S0[2][cc] + 0.5 * DS[1][bb] * S0[2][cc] +
                                            0.5 * S0[1][bb] * DS[2][cc] +
                                            DS[1][bb] * DS[2][cc] / 3.0);
                    acc -= q * wx / dt;
                    *jext_at(b, Jext, 0, nn[0] + a - SW / 2, nn[1] + bb - SW / 2,
                             nn[2] + cc - SW / 2) += acc;
                }
            }
        for (int a = 0; a < SW; a++)
            for (int cc = 0; cc < SW; cc++) {
                double acc = 0.0;
                for (int bb = 0; bb < SW - 1; bb++) {
                    double wy = DS[1][bb] * (S0[0][a] * S0[2][cc] + 0.5 * DS[0][a] * S0[2][cc] +
                                             0.5 * S0[0][a] * DS[2][cc] +
                                             DS[0][a] * DS[2][cc] / 3.0);
                    acc -= q * wy / dt;
                    *jext_at(b, Jext, 1, nn[0] + a - SW / 2, nn[1] + bb - SW / 2,
                             nn[2] + cc - SW / 2) += acc;
                }
            }
        for (int a = 0; a < SW; a++)
            for (int bb = 0; bb < SW; bb++) {
                double acc = 0.0;
                for (int cc = 0; cc < SW - 1; cc++) {
                    double wz = DS[2][cc] * (S0[0][a] * S0[1][bb] + 0.5 * DS[0][a] * S0[1][bb] +
                                             0.5 * S0[0][a] * DS[1][bb] +
                                             DS[0][a] * DS[1][bb] / 3.0);
                    acc -= q * wz / dt;
                    *jext_at(b, Jext, 2, nn[0] + a - SW / 2, nn[1] + bb - SW / 2,
                             nn[2] + cc - SW / 2) += acc;
                }
            }
    } else {
        for (int bb = 0; bb < SW; bb++) {
            double acc = 0.0;
            for (int a = 0; a < SW - 1; a++) {
                double wx = DS[0][a] * (S0[1][bb] + 0.5 * DS[1][bb]);
                acc -= q * wx / dt;
                *jext_at(b, Jext, 0, nn[0] + a - SW / 2, nn[1] + bb - SW / 2, 0) += acc;
            }
        }
        for (int a = 0; a < SW; a++) {
            double acc = 0.0;
            for (int bb = 0; bb < SW - 1; bb++) {
                double wy = DS[1][bb] * (S0[0][a] + 0.5 * DS[0][a]);
                acc -= q * wy / dt;
                *jext_at(b, Jext, 1, nn[0] + a - SW / 2, nn[1] + bb - SW / 2, 0) += acc;
            }
        }
        double vz = dz / dt;
        for (int a = 0; a < SW; a++)
            for (int bb = 0; bb < SW; bb++) {
                double w = S0[0][a] * S0[1][bb] + 0.5 * DS[0][a] * S0[1][bb] +
                           0.5 * S0[0][a] * DS[1][bb] + DS[0][a] * DS[1][bb] / 3.0;
                if (w != 0.0)
                    *jext_at(b, Jext, 2, nn[0] + a - SW / 2, nn[1] + bb - SW / 2, 0) += q * vz * w;
            }
    }
}

void ora_deposit(const ora_box* b, int64_t n, double q, const double* x0, const double* y0,
                 const double* z0, const double* x1, const double* y1, const double* z1,
                 const double* dz, double* Jext)
{
    for (int64_t p = 0; p < n; p++) {
        double X0[3] = {x0[p], y0[p], (b->dim == 3 && z0) ? z0[p] : 0.0};
        double X1[3] = {x1[p], y1[p], (b->dim == 3 && z1) ? z1[p] : 0.0};
        deposit_one(b, q, X0, X1, dz ? dz[p] : 0.0, Jext);
    }
}

/* charge density rho = sum q S(node - X) at the nodes (CIC), periodic */
void ora_charge(const ora_box* b, int64_t n, double q, const double* x, const double* y,
                const double* z, double* rho)
{
    const int nd = b->dim;
    for (int64_t p = 0; p < n; p++) {
        double X[3] = {x[p], y[p], (nd == 3 && z) ? z[p] : 0.0};
        int base[3] = {0, 0, 0};
        double w[3] = {0, 0, 0};
        for (int d = 0; d < nd; d++) {
            double fl = floor(X[d]);
            base[d] = (int)fl;
            w[d] = X[d] - fl;
        }
        for (int c = 0; c < (1 << nd); c++) {
            int ii[3] = {base[0], base[1], base[2]};
            double wt = 1.0;
            for (int d = 0; d < nd; d++) {
                int bit = (c >> d) & 1;
                ii[d] += bit;
                wt *= bit ? w[d] : 1.0 - w[d];
            }
            rho[cidx(b, wrapi(ii[0], b->n[0]), wrapi(ii[1], b->n[1]), wrapi(ii[2], b->n[2]))] +=
                q * wt;
        }
    }
}

/* ------------------------------------------------------------------ */
/* current finalisation                                                */
/* ------------------------------------------------------------------ */

/* Sec. 2.2: J' collected from x' - x^n is J'(x'); J' on the grid of lab coordinates is
   obtained by advecting it along y by v_{s,y} dt/2.  reading: J_lab(x,y) = J_dep(x, y - d),
   d = v_{s,y}(x) dt/2 with v_{s,y} = -s Omega0 x at each component's own x, applied by linear
   interpolation (first-order upwind) on the extended grid; then the x guard columns are
   folded with the shearing-periodic condition at the time of the current, as the transpose
   of the field interpolation.  Other frames fold x periodically. */
void ora_finalize_current(const ora_box* b, const double* Jext, double* J, double t_half)
{
    const int nx = b->n[0], ny = b->n[1], nz = b->n[2];
    const int nxe = nx + 2 * ORA_JG;
    const int64_t ne = jext_cells(b);
    double* T = (double*)malloc(sizeof(double) * 3 * ne);
    memcpy(T, Jext, sizeof(double) * 3 * ne);
    if (sheared(b)) {
        double* tmp = (double*)malloc(sizeof(double) * ny);
        for (int c = 0; c < 3; c++) {
            for (int k = 0; k < nz; k++)
                for (int ie = 0; ie < nxe; ie++) {
                    int i = ie - ORA_JG;
                    double xc = (double)i + STAG_E[c][0] - 0.5 * nx;
                    double d = -b->shear_s * b->omega0 * xc * b->dt / 2.0;
                    double fl = floor(d);
                    int m = (int)fl;
                    double w = d - fl; /* y - d lies between j - m - 1 (weight w) and j - m */
                    for (int j = 0; j < ny; j++) tmp[j] = *jext_at(b, T, c, i, j, k);
                    for (int j = 0; j < ny; j++)
                        *jext_at(b, T, c, i, j, k) =
                            (1.0 - w) * tmp[wrapi(j - m, ny)] + w * tmp[wrapi(j - m - 1, ny)];
                }
        }
        free(tmp);
    }
    const double dys = ora_shear_offset(b, t_half);
    for (int c = 0; c < 3; c++) {
        double* Jc = J + c * ncells(b);
        memset(Jc, 0, sizeof(double) * ncells(b));
        for (int k = 0; k < nz; k++)
            for (int j = 0; j < ny; j++)
                for (int i = 0; i < nx; i++) Jc[cidx(b, i, j, k)] = *jext_at(b, T, c, i, j, k);
        for (int k = 0; k < nz; k++)
            for (int ie = 0; ie < nxe; ie++) {
                int i = ie - ORA_JG;
                if (i >= 0 && i < nx) continue;
                int ii = i >= nx ? i - nx : i + nx;
                for (int j = 0; j < ny; j++) {
                    double v = *jext_at(b, T, c, i, j, k);
                    if (v == 0.0) continue;
                    if (!sheared(b)) {
                        Jc[cidx(b, ii, j, k)] += v;
                    } else {
                        double sh = i >= nx ? dys : -dys;
                        double fl = floor(sh);
                        int js = (int)fl;
                        double w = sh - fl;
                        Jc[cidx(b, ii, wrapi(j + js, ny), k)] += (1.0 - w) * v;
                        Jc[cidx(b, ii, wrapi(j + js + 1, ny), k)] += w * v;
                    }
                }
            }
    }
    free(T);
}

/* ------------------------------------------------------------------ */
/* Maxwell                                                             */
/* ------------------------------------------------------------------ */

/* central curls on the Yee lattice (2D: z derivatives vanish).  Component arrays are read
   through accessors so that boundary conditions and time averages are explicit. */
static double curlE(const ora_box* b, const facc E[3], int c, int i, int j, int k)
{
    const int d3 = b->dim == 3;
    switch (c) {
    case 0: /* at Bx (i, j+1/2, k+1/2): dEz/dy - dEy/dz */
        return (fv(b, &E[2], i, j + 1, k) - fv(b, &E[2], i, j, k)) -
               (d3 ? fv(b, &E[1], i, j, k + 1) - fv(b, &E[1], i, j, k) : 0.0);
    case 1: /* at By (i+1/2, j, k+1/2): dEx/dz - dEz/dx */
        return (d3 ? fv(b, &E[0], i, j, k + 1) - fv(b, &E[0], i, j, k) : 0.0) -
               (fv(b, &E[2], i + 1, j, k) - fv(b, &E[2], i, j, k));
    default: /* at Bz (i+1/2, j+1/2, k): dEy/dx - dEx/dy */
        return (fv(b, &E[1], i + 1, j, k) - fv(b, &E[1], i, j, k)) -
               (fv(b, &E[0], i, j + 1, k) - fv(b, &E[0], i, j, k));
    }
}

static double curlB(const ora_box* b, const facc B[3], int c, int i, int j, int k)
{
    const int d3 = b->dim == 3;
    switch (c) {
    case 0: /* at Ex (i+1/2, j, k): dBz/dy - dBy/dz */
        return (fv(b, &B[2], i, j, k) - fv(b, &B[2], i, j - 1, k)) -
               (d3 ? fv(b, &B[1], i, j, k) - fv(b, &B[1], i, j, k - 1) : 0.0);
    case 1: /* at Ey (i, j+1/2, k): dBx/dz - dBz/dx */
        return (d3 ? fv(b, &B[0], i, j, k) - fv(b, &B[0], i, j, k - 1) : 0.0) -
               (fv(b, &B[2], i, j, k) - fv(b, &B[2], i - 1, j, k));
    default: /* at Ez (i, j, k+1/2): dBy/dx - dBx/dy */
        return (fv(b, &B[1], i, j, k) - fv(b, &B[1], i - 1, j, k)) -
               (fv(b, &B[0], i, j, k) - fv(b, &B[0], i, j - 1, k));
    }
}

static void set_acc(facc* a, const double* F)
{
    a->a = F;
    a->c = NULL;
    a->dys_a = a->dys_c = 0.0;
    a->wa = 1.0;
    a->wc = 0.0;
}

/* Yee leapfrog as B half-step, E full step, B half-step, with the expanding-box scale
   factors of Sec. 3.2: primed fields B' = l L^-1 B, E' = l L^-1 E are advanced with
   L^2 E'/l = L E and L^2 B'/l = L B inside the curls (eq. EBB, EBE), the source is the
   deposited l J', and each field converts back at its own time level.  For the plain and
   leaky frames every factor is 1. */
static void maxwell_leapfrog(ora_box* b, ora_fields* f)
{
    const int nx = b->n[0], ny = b->n[1], nz = b->n[2];
    const int64_t nc = ncells(b);
    const double dt = b->dt;
    const double tn = (double)b->step * dt, th = tn + 0.5 * dt, t1 = tn + dt;
    double ln[3], lh[3], l1[3];
    for (int d = 0; d < 3; d++) {
        ln[d] = ora_scale(b, d, tn);
        lh[d] = ora_scale(b, d, th);
        l1[d] = ora_scale(b, d, t1);
    }
    const double elln = ln[0] * ln[1] * ln[2], ellh = lh[0] * lh[1] * lh[2],
                 ell1 = l1[0] * l1[1] * l1[2];
    double* G = (double*)malloc(sizeof(double) * 3 * nc);  /* L E or L B, the curl argument */
    double* Bp = (double*)malloc(sizeof(double) * 3 * nc); /* B' */
    double* Ep = (double*)malloc(sizeof(double) * 3 * nc); /* E' */
    facc acc[3];
    for (int c = 0; c < 3; c++) set_acc(&acc[c], G + c * nc);

    /* B'^{n+1/2} = B'^n - (dt/2) curl(L^n E^n) */
    for (int c = 0; c < 3; c++)
        for (int64_t q = 0; q < nc; q++) {
            G[c * nc + q] = ln[c] * f->E[c][q];
            Bp[c * nc + q] = elln / ln[c] * f->B[c][q];
        }
#pragma omp parallel for collapse(2)
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++)
                for (int c = 0; c < 3; c++)
                    Bp[c * nc + cidx(b, i, j, k)] -= 0.5 * dt * curlE(b, acc, c, i, j, k);
    /* E'^{n+1} = E'^n + dt curl(L^{n+1/2} B^{n+1/2}) - 4 pi dt (l J') */
    for (int c = 0; c < 3; c++)
        for (int64_t q = 0; q < nc; q++) {
            double Bh = lh[c] / ellh * Bp[c * nc + q];
            G[c * nc + q] = lh[c] * Bh;
            Ep[c * nc + q] = elln / ln[c] * f->E[c][q];
        }
#pragma omp parallel for collapse(2)
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++)
                for (int c = 0; c < 3; c++) {
                    int64_t q = cidx(b, i, j, k);
                    Ep[c * nc + q] += dt * curlB(b, acc, c, i, j, k) - 4.0 * ORA_PI * dt * f->J[c][q];
                }
    for (int c = 0; c < 3; c++)
        for (int64_t q = 0; q < nc; q++) {
            f->E[c][q] = l1[c] / ell1 * Ep[c * nc + q];
            G[c * nc + q] = l1[c] * f->E[c][q];
        }
    /* B'^{n+1} = B'^{n+1/2} - (dt/2) curl(L^{n+1} E^{n+1}) */
#pragma omp parallel for collapse(2)
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++)
                for (int c = 0; c < 3; c++)
                    Bp[c * nc + cidx(b, i, j, k)] -= 0.5 * dt * curlE(b, acc, c, i, j, k);
    for (int c = 0; c < 3; c++)
        for (int64_t q = 0; q < nc; q++) f->B[c][q] = l1[c] / ell1 * Bp[c * nc + q];
    free(G);
    free(Bp);
    free(Ep);
}

/* first-order upwind difference along y of the field seen through acc at (i,j,k) for
   transport velocity w: backward if w > 0, forward otherwise */
static inline double up_dy(const ora_box* b, const facc* a, int i, int j, int k, double w)
{
    return w > 0.0 ? fv(b, a, i, j, k) - fv(b, a, i, j - 1, k)
                   : fv(b, a, i, j + 1, k) - fv(b, a, i, j, k);
}

/* Right-hand sides of eq. (OAB) and eq. (OAE) (Sec. 2.1) with the spatial discretisation of
   Sec. 2.2: central differences on the Yee lattice, first-order upwinding (in the local
   direction of transport) for the advection terms -(v_s.grad)B and +/-(v_s.grad)E'
   ("-" for E'_y, "+" otherwise).  With v_s = v(x) e_y, v = -s Omega0 x:
     dBx/dt  = -(curl E')_x - v dBx/dy
     dBy/dt  = -(curl E')_y - v dBy/dy - s Omega0 Bx
     dBz/dt  = -(curl E')_z - v dBz/dy
     dE'x/dt = (curl B)_x - 4 pi J'x + v dE'x/dy - v dE'y/dx
     dE'y/dt = (curl B)_y - 4 pi J'y - v dE'y/dy - v (dE'x/dx + dE'z/dz)
     dE'z/dt = (curl B)_z - 4 pi J'z + v dE'z/dy - v dE'y/dz
   reading: the non-advective cross derivatives are central and averaged to the target
   component's location; Bx in the tidal term is the 4-point average at By.
   The curls read the fields through Ec, Bc (the combined frame scales them, see maxwell_ksb),
   and kz multiplies v dE'y/dz in dE'z/dt (1 in the shearing box). */
static void ksb_rhs_acc(const ora_box* b, const facc E[3], const facc B[3], const facc Ec[3],
                        const facc Bc[3], double kz, double* const J[3], double* const out[6])
{
    const int nx = b->n[0], ny = b->n[1], nz = b->n[2];
    const int d3 = b->dim == 3;
    const double sO = b->shear_s * b->omega0;
#pragma omp parallel for collapse(2)
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                const int64_t q = cidx(b, i, j, k);
                const double v_int = -sO * ((double)i - 0.5 * nx);        /* at x = i */
                const double v_half = -sO * ((double)i + 0.5 - 0.5 * nx); /* at x = i+1/2 */
                /* Bx at (i, j+1/2, k+1/2) */
                out[0][q] = -curlE(b, Ec, 0, i, j, k) - v_int * up_dy(b, &B[0], i, j, k, v_int);
                /* By at (i+1/2, j, k+1/2) */
                double bx_avg = 0.25 * (fv(b, &B[0], i, j, k) + fv(b, &B[0], i + 1, j, k) +
                                        fv(b, &B[0], i, j - 1, k) + fv(b, &B[0], i + 1, j - 1, k));
                out[1][q] = -curlE(b, Ec, 1, i, j, k) - v_half * up_dy(b, &B[1], i, j, k, v_half) -
                            sO * bx_avg;
                /* Bz at (i+1/2, j+1/2, k) */
                out[2][q] = -curlE(b, Ec, 2, i, j, k) - v_half * up_dy(b, &B[2], i, j, k, v_half);
                /* E'x at (i+1/2, j, k) */
                double dEy_dx = 0.5 * ((fv(b, &E[1], i + 1, j, k) - fv(b, &E[1], i, j, k)) +
                                       (fv(b, &E[1], i + 1, j - 1, k) - fv(b, &E[1], i, j - 1, k)));
                out[3][q] = curlB(b, Bc, 0, i, j, k) - 4.0 * ORA_PI * J[0][q] +
                            v_half * up_dy(b, &E[0], i, j, k, -v_half) - v_half * dEy_dx;
                /* E'y at (i, j+1/2, k) */
                double dEx_dx = 0.5 * ((fv(b, &E[0], i, j, k) - fv(b, &E[0], i - 1, j, k)) +
                                       (fv(b, &E[0], i, j + 1, k) - fv(b, &E[0], i - 1, j + 1, k)));
                double dEz_dz =
                    d3 ? 0.5 * ((fv(b, &E[2], i, j, k) - fv(b, &E[2], i, j, k - 1)) +
                                (fv(b, &E[2], i, j + 1, k) - fv(b, &E[2], i, j + 1, k - 1)))
                       : 0.0;
                out[4][q] = curlB(b, Bc, 1, i, j, k) - 4.0 * ORA_PI * J[1][q] -
                            v_int * up_dy(b, &E[1], i, j, k, v_int) - v_int * (dEx_dx + dEz_dz);
                /* E'z at (i, j, k+1/2) */
                double dEy_dz =
                    d3 ? 0.5 * ((fv(b, &E[1], i, j, k + 1) - fv(b, &E[1], i, j, k)) +
                                (fv(b, &E[1], i, j - 1, k + 1) - fv(b, &E[1], i, j - 1, k)))
                       : 0.0;
                out[5][q] = curlB(b, Bc, 2, i, j, k) - 4.0 * ORA_PI * J[2][q] +
                            v_int * up_dy(b, &E[2], i, j, k, -v_int) - v_int * (kz * dEy_dz);
            }
}

void ora_ksb_rhs(const ora_box* b, double* const E[3], double* const B[3], double dys,
                 double* const J[3], double* const out[6])
{
    facc Ea[3], Ba[3];
    for (int c = 0; c < 3; c++) {
        set_acc(&Ea[c], E[c]);
        set_acc(&Ba[c], B[c]);
        Ea[c].dys_a = Ba[c].dys_a = dys;
    }
    ksb_rhs_acc(b, Ea, Ba, Ea, Ba, 1.0, J, out);
}

void ora_ksb_rhs_f(const ora_box* b, double* const E[3], double* const B[3], double dys,
                   double* const J[3], const double d[3], double kz, double* const out[6])
{
    facc Ea[3], Ba[3], Ec[3], Bc[3];
    for (int c = 0; c < 3; c++) {
        set_acc(&Ea[c], E[c]);
        set_acc(&Ba[c], B[c]);
        Ea[c].dys_a = Ba[c].dys_a = dys;
        Ec[c] = Ea[c];
        Bc[c] = Ba[c];
        Ec[c].wa = Bc[c].wa = d[c];
    }
    ksb_rhs_acc(b, Ea, Ba, Ec, Bc, kz, J, out);
}

/* Sec. 2.2: implicit midpoint in time, F^{n+1} = F^n + dt RHS((F^n + F^{n+1})/2, J'),
   solved by the fixed-point iteration F^{k+1} = F^n + dt RHS((F^n + F^k)/2) from F^0 = F^n.
   reading: a fixed number of iterations (maxwell_iters), or, with maxwell_tol > 0, until
   max|F^{k+1} - F^k| <= tol max|F^{k+1}| (at most maxwell_iters).  The x guards of F^n (and of
   F^0 = F^n) use Delta y_s(t^n), those of every later iterate Delta y_s(t^{n+1}).
   Combined frame (reading): the same step on the expanding-frame fields of Sec. 3.1,
   F'' = (l/l_c) F_c for the c components of E' and B, with the factors of eqs. EBB/EBE at
   t^{n+1/2}: the curls act on (1/l) L^2 F'' (d_c = l_c^2/l), the source is the deposited l J';
   the transport and tidal terms of eqs. OAB/OAE keep their form in the expanding coordinates
   (x and y scale together) except v dE'y/dz in dE'z/dt, which takes kz = (l_y/l_z)^2.  The
   step converts F^n at t^n and F^{n+1} back at t^{n+1}. */
static void maxwell_ksb(ora_box* b, ora_fields* f)
{
    const int64_t nc = ncells(b);
    const double dt = b->dt;
    const double tn = (double)b->step * dt, th = tn + 0.5 * dt, t1 = tn + dt;
    const double dys_n = ora_shear_offset(b, tn), dys_1 = ora_shear_offset(b, t1);
    double sn[3], s1[3], d[3], lh[3];
    for (int c = 0; c < 3; c++) lh[c] = ora_scale(b, c, th);
    {
        double ln[3], l1[3];
        for (int c = 0; c < 3; c++) {
            ln[c] = ora_scale(b, c, tn);
            l1[c] = ora_scale(b, c, t1);
        }
        const double elln = ln[0] * ln[1] * ln[2], ell1 = l1[0] * l1[1] * l1[2];
        const double ellh = lh[0] * lh[1] * lh[2];
        for (int c = 0; c < 3; c++) {
            sn[c] = elln / ln[c];
            s1[c] = ell1 / l1[c];
            d[c] = lh[c] * lh[c] / ellh;
        }
    }
    const double kz = (lh[1] / lh[2]) * (lh[1] / lh[2]);
    double* Fk = (double*)malloc(sizeof(double) * 6 * nc);
    double* Fn = (double*)malloc(sizeof(double) * 6 * nc);
    double* R = (double*)malloc(sizeof(double) * 6 * nc);
    for (int c = 0; c < 3; c++)
        for (int64_t q = 0; q < nc; q++) {
            Fn[c * nc + q] = sn[c] * f->B[c][q];
            Fn[(3 + c) * nc + q] = sn[c] * f->E[c][q];
        }
    memcpy(Fk, Fn, sizeof(double) * 6 * nc);
    double* outp[6];
    for (int c = 0; c < 6; c++) outp[c] = R + c * nc;
    const int maxit = b->maxwell_iters > 0 ? b->maxwell_iters : 8;
    int it;
    for (it = 0; it < maxit; it++) {
        facc Ea[3], Ba[3], Ec[3], Bc[3];
        for (int c = 0; c < 3; c++) {
            Ba[c].a = Fn + c * nc;
            Ba[c].c = Fk + c * nc;
            Ea[c].a = Fn + (3 + c) * nc;
            Ea[c].c = Fk + (3 + c) * nc;
            Ba[c].dys_a = Ea[c].dys_a = dys_n;
            /* F^0 = F^n keeps its own boundary values; later iterates sit at t^{n+1} */
            Ba[c].dys_c = Ea[c].dys_c = it == 0 ? dys_n : dys_1;
            Ba[c].wa = Ba[c].wc = Ea[c].wa = Ea[c].wc = 0.5;
            Ec[c] = Ea[c];
            Bc[c] = Ba[c];
            if (b->frame == ORA_SHEAR_EXPAND) Ec[c].wa = Ec[c].wc = Bc[c].wa = Bc[c].wc = 0.5 * d[c];
        }
        ksb_rhs_acc(b, Ea, Ba, Ec, Bc, b->frame == ORA_SHEAR_EXPAND ? kz : 1.0, f->J, outp);
        double dmax = 0.0, fmax = 0.0;
        for (int64_t q = 0; q < 6 * nc; q++) {
            double nv = Fn[q] + dt * R[q];
            double d = fabs(nv - Fk[q]);
            if (d > dmax) dmax = d;
            if (fabs(nv) > fmax) fmax = fabs(nv);
            Fk[q] = nv;
        }
        if (b->maxwell_tol > 0.0 && dmax <= b->maxwell_tol * fmax) {
            it++;
            break;
        }
    }
    b->last_iters = it;
    for (int c = 0; c < 3; c++)
        for (int64_t q = 0; q < nc; q++) {
            f->B[c][q] = Fk[c * nc + q] / s1[c];
            f->E[c][q] = Fk[(3 + c) * nc + q] / s1[c];
        }
    free(Fk);
    free(Fn);
    free(R);
}

void ora_maxwell(ora_box* b, ora_fields* f)
{
    if (sheared(b))
        maxwell_ksb(b, f);
    else
        maxwell_leapfrog(b, f);
}

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11)                   */
/* ------------------------------------------------------------------ */

void ora_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; r++) {
        uint64_t p0 = (uint64_t)M0 * c0;
        uint64_t p1 = (uint64_t)M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
        k0 += W0;
        k1 += W1;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

void ora_philox_many(int64_t n, const uint32_t* ctr4, const uint32_t* key2, uint32_t* out4)
{
    for (int64_t p = 0; p < n; p++) ora_philox4x32_10(ctr4 + 4 * p, key2 + 2 * p, out4 + 4 * p);
}

/* ------------------------------------------------------------------ */
/* Maxwell-Juttner reinjection sampler                                 */
/* ------------------------------------------------------------------ */

static double mj_density(double u, double theta)
{
    /* isotropic f(u) d^3u proportional to exp(-gamma/theta): density in |u| */
    double g = sqrt(1.0 + u * u);
    return u * u * exp(-(g - 1.0) / theta);
}

/* |u| at which the complementary CDF Q (decreasing, Q[0] = 1, on panels of width h) equals q */
static double mj_quantile(const double* Q, int M, double h, double q)
{
    if (q >= 1.0) return 0.0;
    int lo = 0, hi = M; /* Q[lo] >= q > Q[hi] */
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (Q[mid] >= q)
            lo = mid;
        else
            hi = mid;
    }
    double span = Q[lo] - Q[hi];
    double fr = span > 0 ? (Q[lo] - q) / span : 0.0;
    return (lo + fr) * h;
}

static int log2i(int v)
{
    int b = 0;
    while ((1 << b) < v) b++;
    return b;
}

/* reading (Sec. 4.1 "typically Maxwellian"): Maxwell-Juttner at temperature theta, sampled by
   inverse CDF of |u| from one 32-bit word read as p = w/2^32.  Bulk: table[i] = F^-1(i/nbins),
   i < nbins, linear interpolation in p.  Top bin p >= 1 - 1/nbins: table[nbins-1+k] =
   F^-1(1 - 2^-(b + (32-b) k/ntail)), k = 0..ntail (b = log2 nbins), linear interpolation in
   s = -log2(1-p), where the exponential tail makes the quantile nearly linear.  The CDF comes
   from a Simpson rule on 2^20 panels of [0, u_max], u_max at gamma = 1 + 60 theta. */
void ora_mj_table(double theta, int nbins, int ntail, double* table)
{
    const double gmax = 1.0 + 60.0 * theta;
    const double umax = sqrt(gmax * gmax - 1.0);
    const int M = 1 << 20;
    const double h = umax / M;
    /* complementary CDF summed from the top so that tail probabilities keep full precision */
    double* Q = (double*)malloc(sizeof(double) * (M + 1));
    Q[M] = 0.0;
    for (int k = M - 1; k >= 0; k--) {
        double u0 = k * h;
        Q[k] = Q[k + 1] + h / 6.0 *
                              (mj_density(u0, theta) + 4.0 * mj_density(u0 + 0.5 * h, theta) +
                               mj_density(u0 + h, theta));
    }
    const double tot = Q[0];
    for (int k = 0; k <= M; k++) Q[k] /= tot;
    for (int i = 0; i < nbins; i++) table[i] = mj_quantile(Q, M, h, 1.0 - (double)i / nbins);
    const int bb = log2i(nbins);
    for (int k = 0; k <= ntail; k++) {
        double s = bb + (32.0 - bb) * k / ntail;
        table[nbins - 1 + k] = mj_quantile(Q, M, h, pow(2.0, -s));
    }
    free(Q);
}

/* |u| from w[0] (see ora_mj_table), direction mu = 2U1 - 1, phi = 2 pi U2, U = (w >> 8) 2^-24 */
void ora_mj_sample(const double* table, int nbins, int ntail, const uint32_t w[4], double u[3])
{
    const int bb = log2i(nbins);
    const int sh = 32 - bb;
    const uint32_t bin = w[0] >> sh;
    const uint32_t r = w[0] & ((1u << sh) - 1u);
    double um;
    if ((int)bin < nbins - 1) {
        double fr = (double)r * ldexp(1.0, -sh);
        um = table[bin] + fr * (table[bin + 1] - table[bin]);
    } else {
        /* 1 - p = (2^sh - r) 2^-32, so -log2(1-p) - b = sh - log2(2^sh - r) in [0, sh] */
        double s = (double)sh - log2((double)((1u << sh) - r));
        double x = s * ntail / sh;
        int k = (int)floor(x);
        if (k > ntail - 1) k = ntail - 1;
        double fr = x - k;
        const double* T = table + nbins - 1;
        um = T[k] + fr * (T[k + 1] - T[k]);
    }
    double U1 = (double)(w[1] >> 8) * ldexp(1.0, -24);
    double U2 = (double)(w[2] >> 8) * ldexp(1.0, -24);
    double mu = 2.0 * U1 - 1.0;
    double phi = 2.0 * ORA_PI * U2;
    double st = sqrt(1.0 - mu * mu);
    u[0] = um * st * cos(phi);
    u[1] = um * st * sin(phi);
    u[2] = um * mu;
}

/* ------------------------------------------------------------------ */
/* stable counting sort, tile keys, FP32 offset normalisation          */
/* ------------------------------------------------------------------ */

void ora_stable_sort(int64_t n, const int32_t* keys, int32_t nkeys, int64_t* perm, int64_t* offsets)
{
    int64_t* cnt = (int64_t*)calloc((size_t)nkeys + 2, sizeof(int64_t));
    for (int64_t p = 0; p < n; p++) {
        int32_t k = keys[p];
        if (k < 0 || k > nkeys) k = nkeys;
        cnt[k]++;
    }
    offsets[0] = 0;
    for (int32_t k = 0; k <= nkeys; k++) offsets[k + 1] = offsets[k] + cnt[k];
    for (int32_t k = 0; k <= nkeys; k++) cnt[k] = offsets[k];
    for (int64_t p = 0; p < n; p++) {
        int32_t k = keys[p];
        if (k < 0 || k > nkeys) k = nkeys;
        if (k < nkeys) perm[cnt[k]] = p;
        cnt[k]++;
    }
    free(cnt);
}

void ora_tile_keys(const ora_box* b, const int t[3], int64_t n, const int32_t* ci,
                   const int32_t* cj, const int32_t* ck, int32_t* keys)
{
    const int ntx = (b->n[0] + t[0] - 1) / t[0];
    const int nty = (b->n[1] + t[1] - 1) / t[1];
    const int ntz = (b->n[2] + t[2] - 1) / t[2];
    const int32_t ntiles = ntx * nty * ntz;
    for (int64_t p = 0; p < n; p++) {
        if (ci[p] < 0) {
            keys[p] = ntiles;
            continue;
        }
        int kz = ck ? ck[p] / t[2] : 0;
        keys[p] = ci[p] / t[0] + ntx * (cj[p] / t[1] + nty * kz);
    }
}

/* The FP32 path keeps a position as an int32 cell plus an FP32 offset in [0,1).  After
   s = off + delta (FP32, |delta| < 1): s >= 1 -> (cell+1, s-1), exact for s in [1,2);
   s < 0 -> t = s + 1, (cell-1, t) if t < 1, else (cell, 0) since 1.0 is never stored. */
static float f32_renorm(float off, float delta, int* dc)
{
    volatile float s = off + delta;
    float r = s;
    *dc = 0;
    if (s >= 1.0f) {
        *dc = 1;
        r = s - 1.0f;
    } else if (s < 0.0f) {
        volatile float t = s + 1.0f;
        if (t < 1.0f) {
            *dc = -1;
            r = t;
        } else {
            r = 0.0f;
        }
    }
    return r;
}

void ora_f32_normalize(int64_t n, const int32_t* cell, const float* off, const float* delta,
                       int32_t* cell_out, float* off_out)
{
    for (int64_t p = 0; p < n; p++) {
        int dc;
        off_out[p] = f32_renorm(off[p], delta[p], &dc);
        cell_out[p] = cell[p] + dc;
    }
}

/* The position update of the FP32 path, bit for bit: a particle stored as a cell (linear
   index) plus FP32 in-cell offsets moves by its FP32 deposit displacement D (Sec. 2.2, 3.2,
   4.1).  Per axis the offset takes D in one FP32 addition and is renormalised as above.  The
   shearing box adds its shear move to the y increment (Sec. 2.2): with x^n = (i - n_x/2) +
   off_x the radial coordinate, v_s = -(s Omega0) (x^n + D_x/2) is the flow at the midpoint x
   of the move and dy = D_y + dt v_s, in FP32 with x^n + D_x/2 and D_y + dt v_s each a fused
   multiply-add (one rounding) and s Omega0, dt, n_x/2 cast to FP32 once.  An x-face crossing
   wraps x and, in the shearing box, moves y by +Delta y_s(t^{n+1}) (leaving through x_o) or
   -Delta y_s (through x_i), Sec. 2.1: the FP64 offset splits into floor and an FP32 fraction
   in [0,1) (a fraction that rounds to 1 becomes 0 with the next integer); the fraction is added
   to the y offset and renormalised, the integer to the cell.  y and z wrap periodically.
   err[p] = 1 where a deposit displacement reaches half a cell or the y increment a whole cell
   (the renormalisation then does not apply); the outputs there are not meaningful. */
void ora_f32_move(const ora_box* b, int64_t n, const int32_t* cell, const float* off,
                  const float* disp, int32_t* cell_out, float* off_out, uint8_t* err)
{
    const int nd = b->dim, nx = b->n[0], ny = b->n[1], nz = b->n[2];
    const double t1 = (double)b->step * b->dt + b->dt;
    const double dys = ora_shear_offset(b, t1);
    const double fl = floor(dys);
    int dys_int = (int)fl;
    float dys_frac = (float)(dys - fl);
    if (dys_frac >= 1.0f) {
        dys_frac = 0.0f;
        dys_int = (dys_int + 1) % ny;
    }
    const float sO = (float)(b->shear_s * b->omega0), dt = (float)b->dt;
    const float half_nx = 0.5f * (float)nx;
    for (int64_t p = 0; p < n; p++) {
        int i = cell[p] % nx, j = (cell[p] / nx) % ny, k = cell[p] / (nx * ny);
        float o[3] = {off[p], off[n + p], nd == 3 ? off[2 * n + p] : 0.0f};
        float D[3] = {disp[p], disp[n + p], disp[2 * n + p]};
        float dy = D[1];
        if (sheared(b)) {
            volatile float xr = ((float)i - half_nx) + o[0];
            volatile float mid = fmaf(0.5f, D[0], xr);
            volatile float vs = -sO * mid;
            dy = fmaf(dt, vs, D[1]);
        }
        int bad = !(fabsf(D[0]) < 0.5f && fabsf(D[1]) < 0.5f && (nd == 2 || fabsf(D[2]) < 0.5f) &&
                    fabsf(dy) < 1.0f);
        int dc[3] = {0, 0, 0};
        o[0] = f32_renorm(o[0], D[0], &dc[0]);
        o[1] = f32_renorm(o[1], dy, &dc[1]);
        if (nd == 3) o[2] = f32_renorm(o[2], D[2], &dc[2]);
        i += dc[0];
        j += dc[1];
        k += dc[2];
        if (i >= nx || i < 0) {
            const int out = i >= nx;
            i += out ? -nx : nx;
            if (sheared(b)) {
                int d2;
                o[1] = f32_renorm(o[1], out ? dys_frac : -dys_frac, &d2);
                j += (out ? dys_int : -dys_int) + d2;
            }
        }
        j = wrapi(j, ny);
        if (nd == 3) k = wrapi(k, nz);
        cell_out[p] = (int32_t)cidx(b, i, j, k);
        off_out[p] = o[0];
        off_out[n + p] = o[1];
        if (nd == 3) off_out[2 * n + p] = o[2];
        err[p] = (uint8_t)bad;
    }
}

/* ------------------------------------------------------------------ */
/* one full step                                                       */
/* ------------------------------------------------------------------ */

static inline double wrapd(double v, int n)
{
    double N = (double)n;
    v = fmod(v, N);
    if (v < 0) v += N;
    if (v >= N) v = 0.0;
    return v;
}

/* Per-step scalars of the particle update. */
typedef struct {
    double dt, dys_n, dys_1, sO;
    double lam[3], linv_h[3];
    uint32_t esc_thr;
    double g2thr;
    uint32_t key[2];
} step_scalars;

static void make_scalars(const ora_box* b, step_scalars* S)
{
    const double dt = b->dt;
    const double tn = (double)b->step * dt, th = tn + 0.5 * dt, t1 = tn + dt;
    S->dt = dt;
    S->dys_n = ora_shear_offset(b, tn);
    S->dys_1 = ora_shear_offset(b, t1);
    S->sO = b->shear_s * b->omega0;
    for (int d = 0; d < 3; d++) {
        S->lam[d] = -0.5 * dt * scale_rate(b, d) / ora_scale(b, d, tn); /* Lambda at t^n */
        S->linv_h[d] = 1.0 / ora_scale(b, d, th);                      /* (L^-1)^{n+1/2} */
    }
    S->esc_thr = 0;
    if ((b->frame == ORA_LEAKY || b->escape) && b->leaky_mode == ORA_LEAKY_PROBABILISTIC) {
        double p = b->t_esc > 0 ? dt / b->t_esc : 0.0;
        double th32 = floor(p * 4294967296.0);
        S->esc_thr = th32 >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)th32;
    }
    S->g2thr = b->gamma_thr * b->gamma_thr - 1.0;
    S->key[0] = (uint32_t)b->seed;
    S->key[1] = (uint32_t)(b->seed >> 32);
}

/* One particle of the step orders of Sec. 2.2 (shearing box), Sec. 3.2 (expanding box),
   Sec. 4.1 (leaky box) and standard PIC: gather at x^n -> push -> deposit displacement
   (x' - x^n for the shearing box, the primed displacement for the expanding box, both for the
   combined frame: dt L^-1 u'/gamma'; deposited when Jt is not NULL) -> shear move and
   boundaries -> leaky-box displacement and escape.  In the combined frame the shear move of
   Sec. 2.2 keeps its form in the expanding coordinates (x and y scale together). */
/* One particle's step; returns 1 when the shearing-box effective velocity of the move,
   u'/gamma' + v_s (eq. OAx) with v_s = -s Omega0 x at the midpoint x of the move (the velocity
   the shear move uses), exceeds c = 1: the nonrelativistic velocity transformation allows it
   (Sec. 2.1), and it is counted, not corrected. */
static int particle_update(const ora_box* b, const ora_fields* f, const step_scalars* C,
                           ora_species* S, int64_t p, double* Jt)
{
    int superluminal = 0;
    const int nd = b->dim;
    const int nx = b->n[0];
    const double dt = C->dt;
    double X0[3] = {S->x[p], S->y[p], nd == 3 ? S->z[p] : 0.0};
    double E[3], B[3];
    for (int c = 0; c < 3; c++) {
        E[c] = interp(b, f->E[c], STAG_E[c], X0[0], X0[1], X0[2], C->dys_n);
        B[c] = interp(b, f->B[c], STAG_B[c], X0[0], X0[1], X0[2], C->dys_n);
    }
    double u[3] = {S->ux[p], S->uy[p], S->uz[p]};
    if (b->frame == ORA_SHEAR) {
        double xr = X0[0] - 0.5 * nx;
        ora_push_shear(1, S->q_over_m, dt, b->shear_s, b->omega0, &xr, E, B, u, NULL);
    } else if (b->frame == ORA_SHEAR_EXPAND) {
        double xr = X0[0] - 0.5 * nx;
        ora_push_shear_expand(1, S->q_over_m, dt, b->shear_s, b->omega0, C->lam, b->expand_push,
                              &xr, E, B, u, NULL);
    } else if (b->frame == ORA_EXPAND) {
        ora_push_expand(1, S->q_over_m, dt, C->lam, b->expand_push, E, B, u);
    } else {
        ora_push_boris(1, S->q_over_m, dt, E, B, u);
    }
    const double gam = sqrt(1.0 + dot(u, u));
    double D[3];
    for (int c = 0; c < 3; c++) {
        D[c] = dt * u[c] / gam;
        if (expanding(b)) D[c] *= C->linv_h[c];
    }
    double X1[3] = {X0[0] + D[0], X0[1] + D[1], nd == 3 ? X0[2] + D[2] : 0.0};
    if (Jt) deposit_one(b, S->q, X0, X1, D[2], Jt);
    if (sheared(b)) {
        /* x^{n+1} = x' - s Omega0 (x' + x^n)/2 dt e_y (Sec. 2.2) */
        double xp = X1[0] - 0.5 * nx, xn = X0[0] - 0.5 * nx;
        X1[1] -= C->sO * (xp + xn) / 2.0 * dt;
        const double vs = -C->sO * (xp + xn) / 2.0;
        const double vx = u[0] / gam, vy = u[1] / gam + vs, vz = u[2] / gam;
        superluminal = vx * vx + vy * vy + vz * vz > 1.0;
    }
    if (X1[0] >= nx) {
        X1[0] -= nx;
        if (sheared(b)) X1[1] += C->dys_1;
    } else if (X1[0] < 0.0) {
        X1[0] += nx;
        if (sheared(b)) X1[1] -= C->dys_1;
    }
    X1[0] = wrapd(X1[0], nx);
    X1[1] = wrapd(X1[1], b->n[1]);
    if (nd == 3) X1[2] = wrapd(X1[2], b->n[2]);
    /* the leaky box (Sec. 4.1); in the shearing or expanding frame on request, with the
       displacement D of the deposit (comoving, or primed): the combination the paper's
       conclusion suggests, in this reading */
    if (b->frame == ORA_LEAKY || b->escape) {
        if (b->leaky_mode == ORA_LEAKY_DISPLACEMENT) {
            /* Sec. 4.1: Delta r^n = Delta r^{n-1} + (u/gamma) dt; escape when
               max(|dx|,|dy|) >= l_esc (eq. escape); resample u, reset Delta r.
               reading: u/gamma is the velocity of the push just made. */
            S->drx[p] += D[0];
            S->dry[p] += D[1];
            if (S->drz) S->drz[p] += D[2];
            double m = fmax(fabs(S->drx[p]), fabs(S->dry[p]));
            if (b->use_3vec && S->drz) m = fmax(m, fabs(S->drz[p]));
            if (m >= b->l_esc) {
                uint32_t ctr[4] = {S->id[p], (uint32_t)b->step, 1u, b->box_id}, w[4];
                ora_philox4x32_10(ctr, C->key, w);
                ora_mj_sample(b->mj_table, b->mj_bins, b->mj_tail, w, u);
                S->drx[p] = S->dry[p] = 0.0;
                if (S->drz) S->drz[p] = 0.0;
            }
        } else {
            /* escape with probability dt/t_esc per step above gamma_thr */
            double g2m1 = (u[0] * u[0] + u[1] * u[1]) + u[2] * u[2];
            if (g2m1 > C->g2thr) {
                uint32_t ctr[4] = {S->id[p], (uint32_t)b->step, 0u, b->box_id}, w[4];
                ora_philox4x32_10(ctr, C->key, w);
                if (w[0] < C->esc_thr && S->alive) S->alive[p] = 0;
            }
        }
    }
    S->x[p] = X1[0];
    S->y[p] = X1[1];
    if (nd == 3) S->z[p] = X1[2];
    S->ux[p] = u[0];
    S->uy[p] = u[1];
    S->uz[p] = u[2];
    return superluminal;
}

int ora_particles_only(ora_box* b, const ora_fields* f, ora_species* sp, int nsp)
{
    step_scalars C;
    make_scalars(b, &C);
    for (int s = 0; s < nsp; s++)
        for (int64_t p = 0; p < sp[s].n; p++) {
            if (sp[s].alive && !sp[s].alive[p]) continue;
            b->n_superluminal += particle_update(b, f, &C, &sp[s], p, NULL);
        }
    return 0;
}

/* One full step: the particle updates with deposit, the current finalisation, Maxwell. */
int ora_step(ora_box* b, ora_fields* f, ora_species* sp, int nsp, int nthreads)
{
    step_scalars C;
    make_scalars(b, &C);
    const double th = ((double)b->step + 0.5) * b->dt;
    if (nthreads < 1) nthreads = 1;
#ifdef _OPENMP
    omp_set_num_threads(nthreads);
#else
    nthreads = 1;
#endif
    const int64_t ne = jext_cells(b);
    double* Jbuf = (double*)calloc((size_t)nthreads * 3 * ne, sizeof(double));
    int64_t nsl = 0;
    for (int s = 0; s < nsp; s++) {
        ora_species* S = &sp[s];
#pragma omp parallel num_threads(nthreads)
        {
            int tid = 0;
#ifdef _OPENMP
            tid = omp_get_thread_num();
#endif
            double* Jt = Jbuf + (size_t)tid * 3 * ne;
#pragma omp for schedule(static) reduction(+ : nsl)
            for (int64_t p = 0; p < S->n; p++) {
                if (S->alive && !S->alive[p]) continue;
                nsl += particle_update(b, f, &C, S, p, Jt);
            }
        }
    }
    /* reduce the per-thread current buffers in thread order */
    double* Jext = Jbuf;
    for (int t = 1; t < nthreads; t++)
        for (int64_t q = 0; q < 3 * ne; q++) Jext[q] += Jbuf[(size_t)t * 3 * ne + q];
    double* Jflat = (double*)malloc(sizeof(double) * 3 * ncells(b));
    ora_finalize_current(b, Jext, Jflat, th);
    for (int c = 0; c < 3; c++) memcpy(f->J[c], Jflat + c * ncells(b), sizeof(double) * ncells(b));
    free(Jflat);
    free(Jbuf);
    b->n_superluminal += nsl;
    ora_maxwell(b, f);
    b->step += 1;
    return 0;
}

/* ------------------------------------------------------------------ */
/* diagnostics                                                         */
/* ------------------------------------------------------------------ */

void ora_energies(const ora_box* b, const ora_fields* f, const ora_species* sp, int nsp, double* out)
{
    for (int q = 0; q < 11; q++) out[q] = 0.0;
    const int64_t nc = ncells(b);
    for (int c = 0; c < 3; c++) {
        double se = 0.0, sb = 0.0;
        for (int64_t q = 0; q < nc; q++) {
            se += f->E[c][q] * f->E[c][q];
            sb += f->B[c][q] * f->B[c][q];
        }
        out[c] = se / (8.0 * ORA_PI);
        out[3 + c] = sb / (8.0 * ORA_PI);
    }
    for (int s = 0; s < nsp; s++) {
        const ora_species* S = &sp[s];
        const double m = fabs(S->q / S->q_over_m);
        for (int64_t p = 0; p < S->n; p++) {
            if (S->alive && !S->alive[p]) continue;
            double u[3] = {S->ux[p], S->uy[p], S->uz[p]};
            out[6] += m * (sqrt(1.0 + dot(u, u)) - 1.0);
            out[7] += m * u[0];
            out[8] += m * u[1];
            out[9] += m * u[2];
            out[10] += 1.0;
        }
    }
}
