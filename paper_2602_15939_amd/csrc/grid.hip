// grid.hip — grid kernels of the particle hot path (gfx950): guard fills with the
// shearing-periodic boundary (Sec. 2.1), the current fold with the J' transport along y
// (Sec. 2.2), the Maxwell steps of the three frames (Yee; Yee with the expanding-box scale
// factors of Sec. 3.2; implicit midpoint with upwinded advection solved by fixed-point
// iteration, Sec. 2.2) and the FP64 reductions.
//
// Every grid array carries kGuard guard cells on each side of each axis (z: none in 2D);
// pointers address the interior cell (0,0,0) and the x stride is 1.
#include "pic_internal.h"

namespace pic {

__device__ inline int64_t gidx(const GridDev& G, int x, int y, int z)
{
    return (int64_t)x + (int64_t)G.sy * y + (int64_t)G.sz * z;
}
// i mod n in [0, n); one add or subtract for i in [-n, 2n) (the indices here are within a
// period of the range), the remainder only beyond
__device__ inline int wrapn(int i, int n)
{
    if (i < 0) i += n;
    if (i >= n) i -= n;
    if ((unsigned)i >= (unsigned)n) {
        i %= n;
        if (i < 0) i += n;
    }
    return i;
}

// ------------------------------------------------------------------ guard fill
// Every guard cell takes its value from interior cells: y, z periodic; x periodic, or for the
// shearing box F(x_o + m, y) = F(x_i + m, y + dys) and F(x_i - m, y) = F(x_o - m, y - dys)
// with a fractional dys applied by linear interpolation along y.

// the image of an x guard cell between the two interior values a (at y + js) and b (at
// y + js + 1), weight w on b; the guard fill and the 3D sweep's x halo share it
__device__ inline float shear_lerp(float a, float b, float w) { return fmaf(w, b, (1.f - w) * a); }

// y row offset js and weight w of the image of an x guard cell of the shearing box
// (hi: beyond x = nx - 1, lo: before x = 0): hi y + dys = y + dys_int + w,
// lo y - dys = y - dys_int - 1 + (1 - w)
__device__ inline void shear_image(bool hi, int dys_int, float dys_w, int& js, float& w)
{
    if (hi) {
        js = dys_int;
        w = dys_w;
    } else {
        js = -dys_int - (dys_w > 0.f ? 1 : 0);
        w = dys_w > 0.f ? 1.f - dys_w : 0.f;
    }
}

__device__ __attribute__((always_inline)) inline void fill_guards_body(const FillArgs& a, int blk, int, int c)
{
    const GridDev& G = a.G;
    const int slab = a.slab, shear = a.shear, dys_int = a.dys_int;
    const float dys_w = a.dys_w;
    float* F = a.A.p[c];
    // 32-bit index arithmetic: the x and y guard widths are kGuard, the other divisors are
    // invariant (precomputed multipliers)
    const uint32_t t = (uint32_t)blk * kBlock + threadIdx.x;
    constexpr uint32_t g2 = 2 * kGuard;
    const int gz = G.g[2];
    const uint32_t NYg = (uint32_t)(G.n[1] + 2 * kGuard), NZg = (uint32_t)(G.n[2] + 2 * gz);
    int x, y, z;
    if (slab == 0) {  // x guard slabs over the whole guarded y, z
        if (t >= g2 * NYg * NZg) return;
        const uint32_t m = t % g2, r = t / g2;
        const uint32_t q = G.divyg.div(r);
        y = (int)(r - q * NYg) - kGuard;
        z = (int)q - gz;
        x = (int)m < kGuard ? (int)m - kGuard : G.n[0] + ((int)m - kGuard);
    } else if (slab == 1) {  // y guard slabs over interior x, guarded z
        if (t >= (uint32_t)G.n[0] * g2 * NZg) return;
        const uint32_t r = G.div0.div(t);
        x = (int)(t - r * (uint32_t)G.n[0]);
        const uint32_t m = r % g2;
        z = (int)(r / g2) - gz;
        y = (int)m < kGuard ? (int)m - kGuard : G.n[1] + ((int)m - kGuard);
    } else {  // z guard slabs over interior x, y
        if (t >= (uint32_t)G.n[0] * (uint32_t)G.n[1] * (uint32_t)(2 * gz)) return;
        const uint32_t r = G.div0.div(t);
        x = (int)(t - r * (uint32_t)G.n[0]);
        const uint32_t q = G.div1.div(r);
        y = (int)(r - q * (uint32_t)G.n[1]);
        const int m = (int)q;
        z = m < gz ? m - gz : G.n[2] + (m - gz);
    }
    const int sz_ = wrapn(z, G.n[2]);
    float v;
    if (x < 0 || x >= G.n[0]) {
        const bool hi = x >= G.n[0];
        const int sx = hi ? x - G.n[0] : x + G.n[0];
        if (shear) {
            int js;
            float w;
            shear_image(hi, dys_int, dys_w, js, w);
            const float a = F[gidx(G, sx, wrapn(y + js, G.n[1]), sz_)];
            const float b = F[gidx(G, sx, wrapn(y + js + 1, G.n[1]), sz_)];
            v = shear_lerp(a, b, w);
        } else {
            v = F[gidx(G, sx, wrapn(y, G.n[1]), sz_)];
        }
    } else {
        v = F[gidx(G, x, wrapn(y, G.n[1]), sz_)];
    }
    F[gidx(G, x, y, z)] = v;
}
PIC_BATCHED_KERNEL(fill_guards, FillArgs, kBlock)

// ------------------------------------------------------------------ current fold

// Periodic fold along axis a (1 = y, 2 = z) over the whole guarded extent of the axes before
// it (x and, for z, y) and the interior of the others.
__device__ __attribute__((always_inline)) inline void fold_periodic_body(const FoldPArgs& args, int blk, int, int c)
{
    const GridDev& G = args.G;
    const int a = args.axis;
    float* F = args.J.p[c];
    const int64_t t = (int64_t)blk * kBlock + threadIdx.x;
    const int gx = G.g[0], gy = G.g[1];
    const int NXg = G.n[0] + 2 * gx, NYg = G.n[1] + 2 * gy;
    const int na = G.n[a], ga = G.g[a];
    const int nl = na < 2 * ga ? na : 2 * ga;  // boundary layers that receive
    int x, y, z, m;
    if (a == 2) {
        const int64_t tot = (int64_t)NXg * NYg * nl;
        if (t >= tot) return;
        x = (int)(t % NXg) - gx;
        int64_t r = t / NXg;
        y = (int)(r % NYg) - gy;
        m = (int)(r / NYg);
        z = m < ga ? m : na - (m - ga) - 1;
        if (m >= ga && z < ga) return;  // a small axis: layer already handled
    } else {
        const int64_t tot = (int64_t)NXg * nl * G.n[2];
        if (t >= tot) return;
        x = (int)(t % NXg) - gx;
        int64_t r = t / NXg;
        m = (int)(r % nl);
        z = (int)(r / nl);
        y = m < ga ? m : na - (m - ga) - 1;
        if (m >= ga && y < ga) return;
    }
    const int i = a == 2 ? z : y;
    float v = 0.f;
    int64_t self = gidx(G, x, y, z);
    if (i < ga) v += F[self + (int64_t)na * (a == 2 ? G.sz : G.sy)];
    if (i >= na - ga) v += F[self - (int64_t)na * (a == 2 ? G.sz : G.sy)];
    F[self] += v;
}
PIC_BATCHED_KERNEL(fold_periodic, FoldPArgs, kBlock)

// interior coordinates of linear interior index t = x + n0 (y + n1 z) (below 2^31)
__device__ inline void cell_of(const GridDev& G, int64_t t, int& x, int& y, int& z)
{
    const uint32_t u = (uint32_t)t;
    const uint32_t r = G.div0.div(u);
    x = (int)(u - r * (uint32_t)G.n[0]);
    const uint32_t zz = G.div1.div(r);
    y = (int)(r - zz * (uint32_t)G.n[1]);
    z = (int)zz;
}

// J' at guarded column xg moved along y by v_s(xg) dt/2 (Sec. 2.2), v_s taken at the
// component's staggered x: first-order upwind, i.e. linear interpolation between rows
__device__ inline float shear_transport(const GridDev& G, const float* __restrict__ F, int c, int xg,
                                        int y, int z, float sO_hdt, float half_nx)
{
    const float xc = (float)xg + (c == 0 ? 0.5f : 0.f) - half_nx;
    const float d = -sO_hdt * xc;
    const float fl = floorf(d);
    const int m = (int)fl;
    const float w = d - fl;
    const float fa = F[gidx(G, xg, wrapn(y - m, G.n[1]), z)];
    const float fb = F[gidx(G, xg, wrapn(y - m - 1, G.n[1]), z)];
    return (1.f - w) * fa + w * fb;
}
// The transport and the shearing-periodic x fold in one pass (out-of-place): an interior cell
// takes its own transported value plus, on the first and last g columns, the transported
// guard column of the other face at the y shift of the shearing-periodic map (the exact
// transpose of the field guard fill's interpolation).
__device__ __attribute__((always_inline)) inline void shear_fold_cell(const ShearFoldArgs& a, int64_t t, int c)
{
    const GridDev& G = a.G;
    int x, y, z;
    cell_of(G, t, x, y, z);
    const int nx = G.n[0], ny = G.n[1], ga = G.g[0];
    const float* F = a.in.p[c];
    float v = shear_transport(G, F, c, x, y, z, a.sO_hdt, a.half_nx);
    if (x < ga) {  // guard column x + nx, the image of (x, y + dys)
        v += (1.f - a.dys_w) * shear_transport(G, F, c, x + nx, wrapn(y - a.dys_int, ny), z, a.sO_hdt, a.half_nx) +
             a.dys_w * shear_transport(G, F, c, x + nx, wrapn(y - a.dys_int - 1, ny), z, a.sO_hdt, a.half_nx);
    }
    if (x >= nx - ga) {  // guard column x - nx, the image of (x, y - dys)
        // shift -dys = js + w with js = -dys_int - 1, w = 1 - dys_w (dys_w > 0), else -dys_int
        int js = -a.dys_int;
        float w = 0.f;
        if (a.dys_w > 0.f) {
            js = -a.dys_int - 1;
            w = 1.f - a.dys_w;
        }
        v += (1.f - w) * shear_transport(G, F, c, x - nx, wrapn(y - js, ny), z, a.sO_hdt, a.half_nx) +
             w * shear_transport(G, F, c, x - nx, wrapn(y - js - 1, ny), z, a.sO_hdt, a.half_nx);
    }
    a.out.p[c][gidx(G, x, y, z)] = v;
}
// grid-stride over the cells (the batched launch gives every cell its own thread)
__device__ __attribute__((always_inline)) inline void shear_fold_body(const ShearFoldArgs& a, int blk, int nblk, int c)
{
    const int64_t n = (int64_t)a.G.n[0] * a.G.n[1] * a.G.n[2];
    for (int64_t t = (int64_t)blk * kBlock + threadIdx.x; t < n; t += (int64_t)nblk * kBlock)
        shear_fold_cell(a, t, c);
}
PIC_BATCHED_KERNEL(shear_fold, ShearFoldArgs, kBlock)

// x fold as a gather into interior cells: out(i) = in(i) plus the x guard columns that map
// to i (periodic, or shearing-periodic at dys as the transpose of the guard interpolation).
// Runs over all interior cells when in != out, else over the boundary layers only.
__device__ __attribute__((always_inline)) inline void fold_x_body(const FoldXArgs& a, int blk, int, int c)
{
    const GridDev& G = a.G;
    const Comp3& Jin = a.in;
    const Comp3& Jout = a.out;
    const int all = a.all, shear = a.shear, dys_int = a.dys_int;
    const float dys_w = a.dys_w;
    const int64_t t = (int64_t)blk * kBlock + threadIdx.x;
    const int nx = G.n[0], ga = G.g[0];
    const int nl = all ? nx : (nx < 2 * ga ? nx : 2 * ga);
    const int64_t tot = (int64_t)nl * G.n[1] * G.n[2];
    if (t >= tot) return;
    int m = (int)(t % nl);
    const int64_t r = t / nl;
    const int y = (int)(r % G.n[1]);
    const int z = (int)(r / G.n[1]);
    int x;
    if (all) {
        x = m;
    } else {
        x = m < ga ? m : nx - (m - ga) - 1;
        if (m >= ga && x < ga) return;
    }
    const float* F = Jin.p[c];
    float v = F[gidx(G, x, y, z)];
    if (x < ga) {  // receives guard column x + nx, the image of (x, y + dys)
        if (shear) {
            // guard (nx+x, j) adds (1-w) to (x, j + js) and w to (x, j + js + 1), js = dys_int
            v += (1.f - dys_w) * F[gidx(G, x + nx, wrapn(y - dys_int, G.n[1]), z)] +
                 dys_w * F[gidx(G, x + nx, wrapn(y - dys_int - 1, G.n[1]), z)];
        } else {
            v += F[gidx(G, x + nx, y, z)];
        }
    }
    if (x >= nx - ga) {  // receives guard column x - nx, the image of (x, y - dys)
        if (shear) {
            // shift -dys = js' + w' with js' = -dys_int - 1, w' = 1 - w (w > 0), else -dys_int
            int js = -dys_int;
            float w = 0.f;
            if (dys_w > 0.f) {
                js = -dys_int - 1;
                w = 1.f - dys_w;
            }
            v += (1.f - w) * F[gidx(G, x - nx, wrapn(y - js, G.n[1]), z)] +
                 w * F[gidx(G, x - nx, wrapn(y - js - 1, G.n[1]), z)];
        } else {
            v += F[gidx(G, x - nx, y, z)];
        }
    }
    Jout.p[c][gidx(G, x, y, z)] = v;
}
PIC_BATCHED_KERNEL(fold_x, FoldXArgs, kBlock)

// ------------------------------------------------------------------ Maxwell
// Yee curls (c = 1, dx = 1).  E_j and B_j enter multiplied by ge[j], gb[j] (the l_j of the
// expanding box, 1 otherwise).


// B_i <- fout_i (fin_i B_i - dt/2 curl(g E)_i)
__device__ __attribute__((always_inline)) inline void yee_b_cell(const MaxwellDev& M, int64_t t)
{
    const GridDev& G = M.G;
    int x, y, z;
    cell_of(G, t, x, y, z);
    const int64_t i = gidx(G, x, y, z);
    const int64_t sy = G.sy, sz = G.sz;
    const bool d3 = G.dim == 3;
    const float* Ex = M.E[0];
    const float* Ey = M.E[1];
    const float* Ez = M.E[2];
    const float g0 = M.gf[0], g1 = M.gf[1], g2 = M.gf[2];
    const float cx = g2 * (Ez[i + sy] - Ez[i]) - (d3 ? g1 * (Ey[i + sz] - Ey[i]) : 0.f);
    const float cy = (d3 ? g0 * (Ex[i + sz] - Ex[i]) : 0.f) - g2 * (Ez[i + 1] - Ez[i]);
    const float cz = g1 * (Ey[i + 1] - Ey[i]) - g0 * (Ex[i + sy] - Ex[i]);
    const float h = 0.5f * M.dt;
    M.B[0][i] = M.fout[0] * (M.fin[0] * M.B[0][i] - h * cx);
    M.B[1][i] = M.fout[1] * (M.fin[1] * M.B[1][i] - h * cy);
    M.B[2][i] = M.fout[2] * (M.fin[2] * M.B[2][i] - h * cz);
}
// grid-stride over the cells (the batched launch gives every cell its own thread)
__device__ __attribute__((always_inline)) inline void yee_b_body(const MaxwellDev& M, int blk, int nblk, int)
{
    const int64_t n = (int64_t)M.G.n[0] * M.G.n[1] * M.G.n[2];
    for (int64_t t = (int64_t)blk * kBlock + threadIdx.x; t < n; t += (int64_t)nblk * kBlock) yee_b_cell(M, t);
}
PIC_BATCHED_KERNEL(yee_b, MaxwellDev, kBlock)

// E_i <- fout_i (fin_i E_i + dt curl(g B)_i - 4 pi dt J_i)
__device__ __attribute__((always_inline)) inline void yee_e_cell(const MaxwellDev& M, int64_t t)
{
    const GridDev& G = M.G;
    int x, y, z;
    cell_of(G, t, x, y, z);
    const int64_t i = gidx(G, x, y, z);
    const int64_t sy = G.sy, sz = G.sz;
    const bool d3 = G.dim == 3;
    const float* Bx = M.B[0];
    const float* By = M.B[1];
    const float* Bz = M.B[2];
    const float g0 = M.gf[0], g1 = M.gf[1], g2 = M.gf[2];
    const float cx = g2 * (Bz[i] - Bz[i - sy]) - (d3 ? g1 * (By[i] - By[i - sz]) : 0.f);
    const float cy = (d3 ? g0 * (Bx[i] - Bx[i - sz]) : 0.f) - g2 * (Bz[i] - Bz[i - 1]);
    const float cz = g1 * (By[i] - By[i - 1]) - g0 * (Bx[i] - Bx[i - sy]);
    const float fp = 4.f * 3.14159265358979f * M.dt;
    M.E[0][i] = M.fout[0] * (M.fin[0] * M.E[0][i] + M.dt * cx - fp * M.J[0][i]);
    M.E[1][i] = M.fout[1] * (M.fin[1] * M.E[1][i] + M.dt * cy - fp * M.J[1][i]);
    M.E[2][i] = M.fout[2] * (M.fin[2] * M.E[2][i] + M.dt * cz - fp * M.J[2][i]);
}
// grid-stride over the cells (the batched launch gives every cell its own thread)
__device__ __attribute__((always_inline)) inline void yee_e_body(const MaxwellDev& M, int blk, int nblk, int)
{
    const int64_t n = (int64_t)M.G.n[0] * M.G.n[1] * M.G.n[2];
    for (int64_t t = (int64_t)blk * kBlock + threadIdx.x; t < n; t += (int64_t)nblk * kBlock) yee_e_cell(M, t);
}
PIC_BATCHED_KERNEL(yee_e, MaxwellDev, kBlock)

// FP contraction inside one expression only in the shearing-box sweeps: every kernel that
// computes an iterate (one sweep per launch, two per pass, the face columns of a pass) then
// rounds it the same way, so the paths agree bit for bit.
#pragma clang fp contract(on)

// Shearing box, fixed-point sweeps of the implicit midpoint rule (Sec. 2.2):
//   F^{k+1} = F^n + dt RHS((F^n + F^k)/2, J'),
// RHS of eq. OAB / eq. OAE with v = -s Omega0 x:
//   dB/dt  = -curl E' - v dB/dy (upwind) - s Omega0 <Bx> e_y
//   dE'/dt = curl B - 4 pi J' + (+v dEx/dy, -v dEy/dy, +v dEz/dy) (upwind)
//            - v (dEy/dx, dEx/dx + dEz/dz, dEy/dz) (central, averaged onto the component).
// The field part L of RHS is linear (the upwind side depends only on the sign of v at the
// component), so with C = F^n + dt/2 L(F^n) - 4 pi dt J' (fixed during the step) every sweep is
//   F^{k+1} = C + dt/2 L(F^k).
// The first sweep (F^0 = F^n) also writes C.
//
// The stencil is written once against an accessor V(c, dx, dy, dz) of the iterate.
enum { BX = 0, BY, BZ, EX, EY, EZ };

template <bool D3, class Acc>
__device__ inline void ksb_operator(const Acc& V, float v0, float vh, float sO, float L[6])
{
    // curl E' at the B locations, curl B at the E locations
    const float cEx = (V(EZ, 0, 1, 0) - V(EZ, 0, 0, 0)) - (D3 ? V(EY, 0, 0, 1) - V(EY, 0, 0, 0) : 0.f);
    const float cEy = (D3 ? V(EX, 0, 0, 1) - V(EX, 0, 0, 0) : 0.f) - (V(EZ, 1, 0, 0) - V(EZ, 0, 0, 0));
    const float cEz = (V(EY, 1, 0, 0) - V(EY, 0, 0, 0)) - (V(EX, 0, 1, 0) - V(EX, 0, 0, 0));
    const float cBx = (V(BZ, 0, 0, 0) - V(BZ, 0, -1, 0)) - (D3 ? V(BY, 0, 0, 0) - V(BY, 0, 0, -1) : 0.f);
    const float cBy = (D3 ? V(BX, 0, 0, 0) - V(BX, 0, 0, -1) : 0.f) - (V(BZ, 0, 0, 0) - V(BZ, -1, 0, 0));
    const float cBz = (V(BY, 0, 0, 0) - V(BY, -1, 0, 0)) - (V(BX, 0, 0, 0) - V(BX, 0, -1, 0));
    const float bxa = 0.25f * (V(BX, 0, 0, 0) + V(BX, 1, 0, 0) + V(BX, 0, -1, 0) + V(BX, 1, -1, 0));
    const float dEy_dx = 0.5f * ((V(EY, 1, 0, 0) - V(EY, 0, 0, 0)) + (V(EY, 1, -1, 0) - V(EY, 0, -1, 0)));
    const float dEx_dx = 0.5f * ((V(EX, 0, 0, 0) - V(EX, -1, 0, 0)) + (V(EX, 0, 1, 0) - V(EX, -1, 1, 0)));
    const float dEz_dz =
        D3 ? 0.5f * ((V(EZ, 0, 0, 0) - V(EZ, 0, 0, -1)) + (V(EZ, 0, 1, 0) - V(EZ, 0, 1, -1))) : 0.f;
    const float dEy_dz =
        D3 ? 0.5f * ((V(EY, 0, 0, 1) - V(EY, 0, 0, 0)) + (V(EY, 0, -1, 1) - V(EY, 0, -1, 0))) : 0.f;
    // upwind difference along y for transport velocity w
    auto updy = [&](int c, float w) {
        return w > 0.f ? V(c, 0, 0, 0) - V(c, 0, -1, 0) : V(c, 0, 1, 0) - V(c, 0, 0, 0);
    };
    L[BX] = -cEx - v0 * updy(BX, v0);
    L[BY] = -cEy - vh * updy(BY, vh) - sO * bxa;
    L[BZ] = -cEz - vh * updy(BZ, vh);
    L[EX] = cBx + vh * updy(EX, -vh) - vh * dEy_dx;
    L[EY] = cBy - v0 * updy(EY, v0) - v0 * (dEx_dx + dEz_dz);
    L[EZ] = cBz + v0 * updy(EZ, -v0) - v0 * dEy_dz;
}

// The operator of the combined shearing and expanding frame (reading: the step of Sec. 2.2 on
// the expanding-frame fields of Sec. 3.1): the curls act on (1/l) L^2 F, i.e. d[c] F_c, as in
// eqs. EBB/EBE; the transport and tidal terms keep their form in the expanding coordinates (x
// and y scale together) except v dE'y/dz in dE'z/dt, which takes kz = (l_y/l_z)^2.
template <bool D3, class Acc>
__device__ inline void ksb_operator_f(const Acc& V, float v0, float vh, float sO, const float d[3],
                                      float kz, float L[6])
{
    const float cEx = d[2] * (V(EZ, 0, 1, 0) - V(EZ, 0, 0, 0)) - (D3 ? d[1] * (V(EY, 0, 0, 1) - V(EY, 0, 0, 0)) : 0.f);
    const float cEy = (D3 ? d[0] * (V(EX, 0, 0, 1) - V(EX, 0, 0, 0)) : 0.f) - d[2] * (V(EZ, 1, 0, 0) - V(EZ, 0, 0, 0));
    const float cEz = d[1] * (V(EY, 1, 0, 0) - V(EY, 0, 0, 0)) - d[0] * (V(EX, 0, 1, 0) - V(EX, 0, 0, 0));
    const float cBx = d[2] * (V(BZ, 0, 0, 0) - V(BZ, 0, -1, 0)) - (D3 ? d[1] * (V(BY, 0, 0, 0) - V(BY, 0, 0, -1)) : 0.f);
    const float cBy = (D3 ? d[0] * (V(BX, 0, 0, 0) - V(BX, 0, 0, -1)) : 0.f) - d[2] * (V(BZ, 0, 0, 0) - V(BZ, -1, 0, 0));
    const float cBz = d[1] * (V(BY, 0, 0, 0) - V(BY, -1, 0, 0)) - d[0] * (V(BX, 0, 0, 0) - V(BX, 0, -1, 0));
    const float bxa = 0.25f * (V(BX, 0, 0, 0) + V(BX, 1, 0, 0) + V(BX, 0, -1, 0) + V(BX, 1, -1, 0));
    const float dEy_dx = 0.5f * ((V(EY, 1, 0, 0) - V(EY, 0, 0, 0)) + (V(EY, 1, -1, 0) - V(EY, 0, -1, 0)));
    const float dEx_dx = 0.5f * ((V(EX, 0, 0, 0) - V(EX, -1, 0, 0)) + (V(EX, 0, 1, 0) - V(EX, -1, 1, 0)));
    const float dEz_dz =
        D3 ? 0.5f * ((V(EZ, 0, 0, 0) - V(EZ, 0, 0, -1)) + (V(EZ, 0, 1, 0) - V(EZ, 0, 1, -1))) : 0.f;
    const float dEy_dz =
        D3 ? 0.5f * ((V(EY, 0, 0, 1) - V(EY, 0, 0, 0)) + (V(EY, 0, -1, 1) - V(EY, 0, -1, 0))) : 0.f;
    auto updy = [&](int c, float w) {
        return w > 0.f ? V(c, 0, 0, 0) - V(c, 0, -1, 0) : V(c, 0, 1, 0) - V(c, 0, 0, 0);
    };
    L[BX] = -cEx - v0 * updy(BX, v0);
    L[BY] = -cEy - vh * updy(BY, vh) - sO * bxa;
    L[BZ] = -cEz - vh * updy(BZ, vh);
    L[EX] = cBx + vh * updy(EX, -vh) - vh * dEy_dx;
    L[EY] = cBy - v0 * updy(EY, v0) - v0 * (dEx_dx + dEz_dz);
    L[EZ] = cBz + v0 * updy(EZ, -v0) - v0 * (kz * dEy_dz);
}

// ---- tolerance mode of the sweeps
// a sweep's (largest change, largest value) pair meets the tolerance (a finite change only)
__device__ inline bool ksb_met(const uint32_t* pair, float tol)
{
    const float d = __uint_as_float(pair[0]);
    return d <= tol * __uint_as_float(pair[1]) && d <= 3.4028235e38f;
}
// the sweep before this one met the tolerance: uniform over the grid, tested before any work
__device__ inline bool ksb_skip(const KsbDev& K)
{
    return K.conv && K.k > 0 && ksb_met(K.conv + 2 * (K.k - 1), K.tol);
}
// running maxima of |F^{k+1} - F^k| (NaN -> +inf) and |F^{k+1}|
__device__ inline void ksb_track(float fo, float fk, float& dm, float& fm)
{
    const float d = fabsf(fo - fk);
    dm = d == d ? fmaxf(dm, d) : __int_as_float(0x7f800000);
    fm = fmaxf(fm, fabsf(fo));
}
// workgroup maxima (NT threads, whole waves), one atomic pair per workgroup
template <int NT>
__device__ inline void ksb_reduce(float dm, float fm, uint32_t* pair)
{
    __shared__ float red[2][NT / 64];
    for (int o = 32; o > 0; o >>= 1) {
        dm = fmaxf(dm, __shfl_xor(dm, o, 64));
        fm = fmaxf(fm, __shfl_xor(fm, o, 64));
    }
    const int w = threadIdx.x / 64;
    if (threadIdx.x % 64 == 0) {
        red[0][w] = dm;
        red[1][w] = fm;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int j = 1; j < NT / 64; j++) {
            dm = fmaxf(dm, red[0][j]);
            fm = fmaxf(fm, red[1][j]);
        }
        atomicMax(pair, __float_as_uint(dm));
        atomicMax(pair + 1, __float_as_uint(fm));
    }
}

// output of one cell: FIRST writes C and F^1 from F^n, later sweeps F^{k+1} from C; Fk is
// the iterate at the cell (F^n for the first sweep)
template <bool FIRST>
__device__ inline void ksb_store(const KsbDev& K, int64_t i, const float L[6], const float Fk[6],
                                 float& dm, float& fm)
{
    const float h = 0.5f * K.dt;
    const float fpdt = 4.f * 3.14159265358979f * K.dt;
#pragma unroll
    for (int c = 0; c < 6; c++) {
        float Cv;
        if (FIRST) {
            Cv = Fk[c] + h * L[c];
            if (c >= EX) Cv -= fpdt * K.J[c - EX][i];
            K.C[c][i] = Cv;
        } else {
            Cv = K.C[c][i];
        }
        const float v = Cv + h * L[c];
        K.Fo[c][i] = v;
        ksb_track(v, Fk[c], dm, fm);
    }
}

// 2D (and any size): one thread per cell, neighbours straight from memory
template <bool FIRST>
__device__ __attribute__((always_inline)) inline void ksb_sweep_body(const KsbDev& K, int blk, int, int)
{
    if (ksb_skip(K)) return;
    const GridDev& G = K.G;
    const int64_t t = (int64_t)blk * kBlock + threadIdx.x;
    float dm = 0.f, fm = 0.f;
    if (t < (int64_t)G.n[0] * G.n[1] * G.n[2]) {
        int x, y, z;
        cell_of(G, t, x, y, z);
        const int64_t i = gidx(G, x, y, z);
        const int64_t sy = G.sy, sz = G.sz;
        const float* const* F = K.Fk;
        auto V = [&](int c, int dx, int dy, int dz) { return F[c][i + dx + sy * dy + sz * dz]; };
        const float v0 = -K.sO * ((float)x - K.half_nx);         // at x = i
        const float vh = -K.sO * ((float)x + 0.5f - K.half_nx);  // at x = i + 1/2
        float L[6], Fk[6];
        if (K.expand) {
            if (G.dim == 3)
                ksb_operator_f<true>(V, v0, vh, K.sO, K.dfac, K.kz, L);
            else
                ksb_operator_f<false>(V, v0, vh, K.sO, K.dfac, K.kz, L);
        } else if (G.dim == 3) {
            ksb_operator<true>(V, v0, vh, K.sO, L);
        } else {
            ksb_operator<false>(V, v0, vh, K.sO, L);
        }
#pragma unroll
        for (int c = 0; c < 6; c++) Fk[c] = F[c][i];
        ksb_store<FIRST>(K, i, L, Fk, dm, fm);
    }
    if (K.conv) ksb_reduce<kBlock>(dm, fm, K.conv + 2 * K.k);
}
__device__ __attribute__((always_inline)) inline void ksb_first_body(const KsbDev& K, int blk, int n, int y) { ksb_sweep_body<true>(K, blk, n, y); }
__device__ __attribute__((always_inline)) inline void ksb_next_body(const KsbDev& K, int blk, int n, int y) { ksb_sweep_body<false>(K, blk, n, y); }
PIC_BATCHED_KERNEL(ksb_first, KsbDev, kBlock)
PIC_BATCHED_KERNEL(ksb_next, KsbDev, kBlock)

// 3D: a workgroup owns a KX x KY column tile and marches over a chunk of KZ planes; three
// consecutive planes of the iterate (tile plus a one-cell halo) sit in LDS.  Halo positions
// outside the interior are read through the boundary maps of the guard fill (y, z periodic;
// x shearing-periodic with the fractional shift interpolated along y, the same arithmetic), so
// the iterates need no guard fill between sweeps (only the last one's guards are filled, for
// the push).  128 x 4 columns of 64-plane chunks (512 threads, 56 KB of LDS, two workgroups
// per CU) measured fastest at 256^3 among 32..128 x 2..16 x 16..128 (8 % below 32 x 8 x 32).  The iterate written and C read once per sweep use
// nontemporal (streaming) stores and loads: a sweep moves far more than the caches hold, and
// the halo reads of the iterate, which neighbouring workgroups share, keep the normal policy
// (another 9 %).
constexpr int KX = 128, KY = 4, KZ = 64;
constexpr int KXH = KX + 2, KYH = KY + 2;

template <bool FIRST>
__global__ __launch_bounds__(KX * KY) void ksb_sweep3_kernel(KsbDev K)
{
    constexpr int NT = KX * KY;
    // staged plane positions: the KX tile columns of the KYH rows, then the 2 * KYH x halo
    // positions, two per thread: j = 0 covers the first NT column positions, j = 1 the rest
    // and the x halo (the grid's x size is a multiple of KX, so only these can be x halo)
    constexpr int NCOL = KX * KYH, NPOS = NCOL + 2 * KYH;
    static_assert(NCOL >= NT && NPOS <= 2 * NT, "two staged positions per thread");
    __shared__ float P[3][6][KYH * KXH];
    if (ksb_skip(K)) return;
    const GridDev& G = K.G;
    const int tid = threadIdx.x, tx = tid % KX, ty = tid / KX;
    // tiles x fastest, then y, then z chunk; each XCD takes a contiguous range so that the
    // halos of neighbouring tiles are shared in its L2
    const int nx = G.n[0], ny = G.n[1], nz = G.n[2];
    const int ntx = nx / KX, nty = (ny + KY - 1) / KY;
    const int tile = xcd_contiguous(blockIdx.x, gridDim.x);
    const int x0 = (tile % ntx) * KX, y0 = ((tile / ntx) % nty) * KY, z0 = (tile / (ntx * nty)) * KZ;
    const int z1 = min(z0 + KZ, nz);
    const int x = x0 + tx, y = y0 + ty;
    const bool inside = y < ny;
    const float* const* F = K.Fk;
    // staged position j: LDS slot and in-plane offset of its source.  y and z halo positions
    // are read at their periodic images; the x halo positions (x = -1, x = nx) at their
    // shearing-periodic images: two interior values of the opposite x face, y rows js and
    // js + 1 from the position's y, interpolated as the guard fill does, so that no guard fill
    // is needed between sweeps.  Rows beyond the first one outside the grid (ragged y tiles)
    // are never read by a valid cell.
    int slot[2], off[2];
    bool ok[2];
    bool xh = false;  // position j = 1 is an x halo image
    int off2 = 0;
    float wx = 0.f;
#pragma unroll
    for (int j = 0; j < 2; j++) {
        const int q = tid + j * NT;
        int lx, ly;
        if (q < NCOL) {
            lx = 1 + q % KX;
            ly = q / KX;
        } else {
            const int r = q - NCOL;
            lx = (r & 1) ? KXH - 1 : 0;
            ly = r >> 1;
        }
        const int gx = x0 - 1 + lx, gy = y0 - 1 + ly;
        ok[j] = q < NPOS && gy <= ny;
        slot[j] = ly * KXH + lx;
        int js = 0;
        float w = 0.f;
        const bool img = j == 1 && ok[j] && (gx < 0 || gx >= nx);
        if (img) shear_image(gx >= nx, K.ydys_int, K.ydys_w, js, w);
        const int sx = gx < 0 ? gx + nx : (gx >= nx ? gx - nx : gx);
        const int ya = wrapn(gy + js, ny);
        off[j] = ok[j] ? sx + G.sy * ya : 0;
        if (j == 1) {
            xh = img;
            off2 = img ? sx + G.sy * wrapn(ya + 1, ny) : 0;
            wx = w;
        }
    }
    // register stage of one plane (loads in flight while the previous plane is computed; the
    // x images are interpolated when the plane is stashed)
    float R[2][6], R2[6];
    auto fetch = [&](int z) {
        const int64_t pz = (int64_t)G.sz * (z < 0 ? z + nz : (z >= nz ? z - nz : z));
#pragma unroll
        for (int c = 0; c < 6; c++) {
            R[0][c] = ok[0] ? F[c][off[0] + pz] : 0.f;
            R[1][c] = ok[1] ? F[c][off[1] + pz] : 0.f;
            R2[c] = xh ? F[c][off2 + pz] : 0.f;
        }
    };
    auto stash = [&](int s) {
#pragma unroll
        for (int c = 0; c < 6; c++) {
            if (ok[0]) P[s][c][slot[0]] = R[0][c];
            if (ok[1]) P[s][c][slot[1]] = xh ? shear_lerp(R[1][c], R2[c], wx) : R[1][c];
        }
    };
    const float v0 = -K.sO * ((float)x - K.half_nx);
    const float vh = -K.sO * ((float)x + 0.5f - K.half_nx);
    fetch(z0 - 1);
    stash(0);
    fetch(z0);
    stash(1);
    fetch(z0 + 1);
    int sm = 0, sc = 1, sp = 2;
    const int c0 = (ty + 1) * KXH + (tx + 1);
    const int64_t i0 = gidx(G, x, y, 0);
    float dm = 0.f, fm = 0.f;
    for (int z = z0; z < z1; z++) {
        stash(sp);                   // plane z+1
        if (z + 2 <= z1) fetch(z + 2);  // in flight during this plane
        float Cv[6];
        const int64_t i = i0 + (int64_t)G.sz * z;
        if (!FIRST && inside)
#pragma unroll
            for (int c = 0; c < 6; c++) Cv[c] = __builtin_nontemporal_load(&K.C[c][i]);
        __syncthreads();
        auto V = [&](int c, int dx, int dy, int dz) {
            const int slot = dz < 0 ? sm : (dz > 0 ? sp : sc);
            return P[slot][c][c0 + dx + KXH * dy];
        };
        if (inside) {
            float L[6];
            ksb_operator<true>(V, v0, vh, K.sO, L);
            const float h = 0.5f * K.dt;
            if (FIRST) {
                const float fpdt = 4.f * 3.14159265358979f * K.dt;
#pragma unroll
                for (int c = 0; c < 6; c++) {
                    float cv = P[sc][c][c0] + h * L[c];
                    if (c >= EX) cv -= fpdt * K.J[c - EX][i];
                    __builtin_nontemporal_store(cv, &K.C[c][i]);
                    const float v = cv + h * L[c];
                    __builtin_nontemporal_store(v, &K.Fo[c][i]);
                    if (K.conv) ksb_track(v, P[sc][c][c0], dm, fm);
                }
            } else {
#pragma unroll
                for (int c = 0; c < 6; c++) {
                    const float v = Cv[c] + h * L[c];
                    __builtin_nontemporal_store(v, &K.Fo[c][i]);
                    if (K.conv) ksb_track(v, P[sc][c][c0], dm, fm);
                }
            }
        }
        __syncthreads();
        const int t = sm;
        sm = sc;
        sc = sp;
        sp = t;
    }
    if (K.conv) ksb_reduce<NT>(dm, fm, K.conv + 2 * K.k);
}

// ---- two sweeps per pass (3D, fixed sweep count)
// A pass takes F^k to F^{k+2} = C + dt/2 L(F^{k+1}) with F^{k+1} = C + dt/2 L(F^k) kept in LDS:
// the workgroup computes F^{k+1} on its PX x PY tile plus a one-cell halo, from F^k on the tile
// plus a two-cell halo, then F^{k+2} on the tile, marching over z with three planes of each
// iterate in LDS.  Memory sees one read of F^k and C and one write of F^{k+2} for two sweeps
// (the first pass reads F^n and J and writes C and F^2).
// The x halo of F^{k+1} beyond a shearing-periodic face is an image of the opposite face's
// F^{k+1} at another y, which another workgroup owns: a face tile recomputes those values
// itself, from F^k on the opposite face's three columns (one of them an image again) over the
// rows the image interpolates between, one plane ahead of its own F^{k+1}.
// Every value is the same expression as in the one-sweep kernels (contraction inside one
// expression only), so a pass gives the two sweeps' iterate bit for bit.
// Pipeline per plane: the stores of the previous plane's results, then the loads for the
// next plane (F^k and C in two alternating register sets), which nothing reads before the
// next plane, so the loads of a whole plane overlap the computation.
// Roles: every thread stages one F^k column position (the PY + 4 window rows over the PX tile
// columns); the threads of the first PY + 2 rows compute F^{k+1} on the window rows, those of
// rows 1..PY also F^{k+2} on the tile; wave WXA stages the x-halo columns of F^k, WXB computes
// the x-halo columns of F^{k+1}, WO0 and WO1 stage the opposite-face columns of F^k (one side
// each), WAUX computes the opposite-face values of F^{k+1}.
template <int X>
struct PassTile {
    static constexpr int PX = X, PY = 4, PZ = 64;
    static constexpr int W0X = PX + 4, W0Y = PY + 4;  // F^k window: tile + 2 (x from x0 - 2, y from y0 - 2)
    static constexpr int W1X = PX + 2, W1Y = PY + 2;  // F^{k+1} window: tile + 1
    static constexpr int XR1 = W1Y + 1, XR0 = XR1 + 2;  // opposite-face rows of F^{k+1} and of F^k
    static constexpr int PN = W0Y * PX;                 // one staged F^k position per thread
    // the extra roles go to the waves past the window rows where there are some (a 1024-thread
    // tile), else to the two last waves, which also compute (a 512-thread tile)
    static constexpr int WXA = 0, WXB = W1Y * PX / 64;
    static constexpr int WO0 = PN == 1024 ? 13 : WXB, WO1 = PN == 1024 ? 15 : WXB + 1;
    static constexpr int WAUX = PN == 1024 ? 14 : WXB + 1;
};
// 64 x 4 tiles: 512 threads and 72 KB of LDS, two workgroups per CU.  At 256^3 a pass takes
// 0.44 ms, the same as the 128 x 4 tile (1024 threads, 137 KB, one workgroup per CU), against
// 0.49 ms for two single sweeps.  Neither the stencil (the pass without it takes as long) nor
// HBM bandwidth bounds it: the loads of one plane, one plane ahead, are its memory parallelism,
// and a second register set for two planes ahead spills (measured slower).
constexpr int kPassX = 64;

// element of an array at a 32-bit byte offset from its base (the array pointer itself, in
// scalar registers): plane and in-plane offsets are summed in 32 bits, so the compiler keeps
// one offset register per position instead of a 64-bit address per array (the arrays of a
// box that takes the pass span less than 4 GiB)
__device__ inline float ld_off(const float* base, uint32_t ob)
{
    return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(base) + ob);
}
__device__ inline float* st_off(float* base, uint32_t ob)
{
    return reinterpret_cast<float*>(reinterpret_cast<char*>(base) + ob);
}

template <int TX, bool FIRST>
__global__ __launch_bounds__(PassTile<TX>::PN) __attribute__((amdgpu_waves_per_eu(4)))
void ksb_pass3_kernel(KsbDev K)
{
    using T = PassTile<TX>;
    constexpr int PX = T::PX, PY = T::PY, PZ = T::PZ, PN = T::PN;
    constexpr int W0X = T::W0X, W0Y = T::W0Y, W1X = T::W1X, W1Y = T::W1Y, XR0 = T::XR0, XR1 = T::XR1;
    static_assert(PX % 64 == 0 && W1Y * PX == 64 * T::WXB && T::WAUX < PN / 64 && T::WO1 < PN / 64,
                  "thread roles");
    static_assert(2 * W1Y <= 64 && PX + PY * PX <= 64 * T::WXB, "F^{k+2} on window-row waves");
    static_assert(3 * XR0 <= 32 && XR1 <= 32, "opposite-face roles fit half a wave per side");
    __shared__ float A[3][6][W0Y * W0X];  // planes of F^k
    __shared__ float Bs[3][6][W1Y * W1X];  // planes of F^{k+1}
    __shared__ float XA[3][2][6][3 * XR0];  // opposite-face F^k: [plane][side][c][row * 3 + col]
    __shared__ float XB[2][2][6][XR1];      // opposite-face F^{k+1}: [plane][side][c][row]
    const GridDev& G = K.G;
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
    const int nx = G.n[0], ny = G.n[1], nz = G.n[2];
    const int ntx = nx / PX, nty = (ny + PY - 1) / PY;
    const int tile = xcd_contiguous(blockIdx.x, gridDim.x);
    const int x0 = (tile % ntx) * PX, y0 = ((tile / ntx) % nty) * PY, z0 = (tile / (ntx * nty)) * PZ;
    const int z1 = min(z0 + PZ, nz);
    const float* const* F = K.Fk;
    const float h = 0.5f * K.dt;
    const float fpdt = 4.f * 3.14159265358979f * K.dt;
    // side 0: the face at x = 0 (x halo x = -1, an image of column nx - 1); side 1: x = nx - 1
    const bool face[2] = {x0 == 0, x0 + PX == nx};
    int js1[2];
    float w1[2];
    shear_image(false, K.y1_int, K.y1_w, js1[0], w1[0]);
    shear_image(true, K.y1_int, K.y1_w, js1[1], w1[1]);

    // ---- staged F^k position of every thread: window row tid / PX, tile column tid % PX
    const uint32_t aoff = 4u * (uint32_t)(x0 + tid % PX + G.sy * wrapn(y0 - 2 + tid / PX, ny));
    const int aslot = tid + (W0X - PX) * (tid / PX) + 2;
    // extra F^k position, lanes 0..31 of wave 0 (x-halo columns lx = 0, 1, W0X-2, W0X-1 of
    // F^k) and of waves WO0 and WO1 (column col, row r of the XR0 opposite-face rows of side 0 and
    // side 1).  An image position interpolates two values (shift ydys of F^k): lane l + 32
    // loads the second one for lane l.
    uint32_t xoff = 0;
    int xslot = 0;
    bool xa = false, ximg = false;
    float xw = 0.f;
    const int xs = wv == T::WO1 ? 1 : 0;
    const bool owave = wv == T::WO0 || wv == T::WO1;
    {
        const int l = lane & 31;
        int gx = 0, gy = 0;
        bool pos = false;
        if (wv == T::WXA && l < 4 * W0Y) {
            const int ly = l >> 2, e = l & 3;
            const int lx = e < 2 ? e : W0X - 4 + e;
            gx = x0 - 2 + lx;
            gy = y0 - 2 + ly;
            pos = gx >= -1 && gx <= nx;  // x = -2, nx + 1 beyond a face are never read
            xslot = ly * W0X + lx;
        } else if (owave && l < 3 * XR0) {
            const int col = l % 3, r = l / 3;
            gx = (xs == 0 ? nx - 2 : -1) + col;
            gy = y0 - 2 + js1[xs] + r;
            pos = face[xs];
            xslot = r * 3 + col;
        }
        int js = 0;
        ximg = pos && (gx < 0 || gx >= nx);
        if (ximg) shear_image(gx >= nx, K.ydys_int, K.ydys_w, js, xw);
        const int sx = gx < 0 ? gx + nx : (gx >= nx ? gx - nx : gx);
        const int ya = wrapn(gy + js, ny);
        const bool second = lane >= 32;
        xa = pos && (!second || ximg);  // this lane loads a value
        xoff = xa ? 4u * (uint32_t)(sx + G.sy * (second ? wrapn(ya + 1, ny) : ya)) : 0u;
        if (second) xa = xa && ximg;
        if (second) ximg = false;
        if (second) pos = false;
        xslot = pos ? xslot : -1;  // the lanes that store (lanes < 32 with a position)
    }

    // ---- F^{k+1} position: threads < W1Y * PX on the window rows over the tile columns
    const bool bmain = tid < W1Y * PX;
    const int blx = 1 + tid % PX, bly = bmain ? tid / PX : 0;
    const int bslot = bly * W1X + blx;
    const int bgx = x0 + tid % PX;
    const uint32_t boff = 4u * (uint32_t)(bgx + G.sy * wrapn(y0 - 1 + bly, ny));
    // extra F^{k+1} position (wave WXB: the x-halo columns lx = 0, W1X - 1, rows r >> 1 --
    // interior, or beyond a face an image of the opposite face's values; wave WAUX: row r of the
    // opposite face of side cs, one plane ahead)
    int cslot = 0, cs = 0, crow = 0, cgx = 0;
    bool cop = false, cimg = false, caux = false;
    uint32_t coff = 0;
    if (wv == T::WXB && lane < 2 * W1Y) {
        const int ly = lane >> 1, lx = (lane & 1) ? W1X - 1 : 0;
        cgx = x0 - 1 + lx;
        const int gy = y0 - 1 + ly;
        cslot = ly * W1X + lx;
        crow = ly;
        cimg = cgx < 0 || cgx >= nx;
        cop = !cimg;
        cs = cgx < 0 ? 0 : 1;
        coff = cop ? 4u * (uint32_t)(cgx + G.sy * wrapn(gy, ny)) : 0u;
    }
    if (wv == T::WAUX && (lane & 31) < XR1) {
        cs = lane >> 5;
        crow = lane & 31;
        caux = face[cs];
        cgx = cs == 0 ? nx - 1 : 0;
        coff = caux ? 4u * (uint32_t)(cgx + G.sy * wrapn(y0 - 1 + js1[cs] + crow, ny)) : 0u;
    }
    const bool cload = cop || caux;

    // ---- F^{k+2}: the tile cell of threads PX .. PX + PY * PX - 1 (their F^{k+1} position)
    const bool tmain = tid >= PX && tid < PX + PY * PX;
    const int ty = tid / PX - 1;
    const bool inside = tmain && y0 + ty < ny;
    const uint32_t i0 = 4u * (uint32_t)(bgx + G.sy * min(y0 + max(ty, 0), ny - 1));

    // C of the F^{k+1} positions in two register sets used on alternate planes: the loads
    // for plane q + 1 are issued at the top of plane q, beside the F^k loads
    float R[6], X[6], Ca[6], Cb[6], Cn[6], Ct[6], Ores[6];
#pragma unroll
    for (int c = 0; c < 6; c++) X[c] = Ca[c] = Cb[c] = Cn[c] = Ct[c] = Ores[c] = 0.f;
    auto plane_of = [&](int z) { return 4u * (uint32_t)G.sz * (uint32_t)wrapn(z, nz); };
    auto fetch_main = [&](int z) {
        const uint32_t pz = plane_of(z);
#pragma unroll
        for (int c = 0; c < 6; c++) R[c] = ld_off(F[c], pz + aoff);
        if (wv == T::WXA && xa)
#pragma unroll
            for (int c = 0; c < 6; c++) X[c] = ld_off(F[c], pz + xoff);
    };
    auto fetch_aux = [&](int z) {
        const uint32_t pz = plane_of(z);
        if (owave && xa)
#pragma unroll
            for (int c = 0; c < 6; c++) X[c] = ld_off(F[c], pz + xoff);
    };
    // the extra value of a lane, interpolated with lane + 32's for an image (whole wave)
    auto extra = [&](int c) {
        const float v2 = __shfl(X[c], (lane & 31) + 32, 64);
        return ximg ? shear_lerp(X[c], v2, xw) : X[c];
    };
    auto stash_main = [&](int s) {
#pragma unroll
        for (int c = 0; c < 6; c++) A[s][c][aslot] = R[c];
        if (wv == T::WXA)
#pragma unroll
            for (int c = 0; c < 6; c++) {
                const float v = extra(c);
                if (xslot >= 0) A[s][c][xslot] = v;
            }
    };
    auto stash_aux = [&](int s) {
        if (owave)
#pragma unroll
            for (int c = 0; c < 6; c++) {
                const float v = extra(c);
                if (xslot >= 0) XA[s][xs][c][xslot] = v;
            }
    };
    // C (first pass: J) of the F^{k+1} positions into Cd: main ones and wave WXB's at plane zm,
    // wave WAUX's at za
    auto load_c = [&](float* Cd, int zm, int za) {
        const uint32_t pm = plane_of(zm);
        const uint32_t o = bmain ? boff : coff;
        const uint32_t pc = caux ? plane_of(za) : pm;
        if (bmain || cload)
#pragma unroll
            for (int c = 0; c < 6; c++)
                if (!FIRST || c >= EX)
                    Cd[c] = FIRST ? ld_off(K.J[c - EX], pc + o) : ld_off(K.C[c], pc + o);
    };
    // F^{k+1} = C + dt/2 L(F^k) at one position, the operator read through V; the first pass
    // also gives C there (cout)
    auto next_iterate = [&](auto&& V, int gx, const float* cw, float* out, float* cout) {
        const float v0 = -K.sO * ((float)gx - K.half_nx);
        const float vh = -K.sO * ((float)gx + 0.5f - K.half_nx);
        float L[6];
        ksb_operator<true>(V, v0, vh, K.sO, L);
#pragma unroll
        for (int c = 0; c < 6; c++) {
            if (FIRST) {
                float cv = V(c, 0, 0, 0) + h * L[c];
                if (c >= EX) cv -= fpdt * cw[c];
                cout[c] = cv;
                out[c] = cv + h * L[c];
            } else {
                out[c] = cw[c] + h * L[c];
            }
        }
    };
    // opposite-face F^{k+1} at plane z from the opposite-face F^k planes (m, c, p)
    auto aux_iterate = [&](const float* cw, int m, int c0, int p, int xb) {
        if (!caux) return;
        auto V = [&](int c, int dx, int dy, int dz) {
            const int s = dz < 0 ? m : (dz > 0 ? p : c0);
            return XA[s][cs][c][(crow + 1 + dy) * 3 + 1 + dx];
        };
        float out[6], cv[6];
        next_iterate(V, cgx, cw, out, cv);
#pragma unroll
        for (int c = 0; c < 6; c++) XB[xb][cs][c][crow] = out[c];
    };

    // ---- prologue: F^k planes z0 - 2, z0 - 1 (opposite face: z0 - 2 .. z0), the opposite
    // face's F^{k+1} at z0 - 1, then the loads for the first plane
    fetch_main(z0 - 2);
    fetch_aux(z0 - 2);
    stash_main(0);
    stash_aux(0);
    fetch_main(z0 - 1);
    fetch_aux(z0 - 1);
    stash_main(1);
    stash_aux(1);
    fetch_aux(z0);
    load_c(Cb, z0 - 1, z0 - 1);
    stash_aux(2);
    __syncthreads();
    aux_iterate(Cb, 0, 1, 2, 0);
    __syncthreads();  // slot 0 of the opposite-face F^k is staged again at the first plane
    fetch_main(z0);
    fetch_aux(z0 + 1);
    load_c(Ca, z0 - 1, z0);
    int am = 0, ac = 1, ap = 2;  // F^k planes q - 1, q, q + 1
    int bm = 0, bc = 1, bp = 2;  // F^{k+1} planes q - 2, q - 1, q
    int xm = 1, xc = 2, xp = 0;  // opposite-face F^k planes q, q + 1, q + 2
    int xbq = 0;                 // opposite-face F^{k+1} plane q (the other slot: q + 1)
    // one plane: F^{k+1} at q with the C set Cu (loaded a plane earlier), the loads of the
    // next plane's C into Cl
    auto plane = [&](int q, float* Cu, float* Cl) {
        stash_main(ap);  // F^k plane q + 1
        stash_aux(xp);   // opposite-face F^k plane q + 2
        if (inside) {
            if (q - 2 >= z0) {
                const uint32_t pz = plane_of(q - 2);
#pragma unroll
                for (int c = 0; c < 6; c++) __builtin_nontemporal_store(Ores[c], st_off(K.Fo[c], pz + i0));
            }
            if (FIRST && q - 1 >= z0 && q - 1 < z1) {
                const uint32_t pz = plane_of(q - 1);
#pragma unroll
                for (int c = 0; c < 6; c++) __builtin_nontemporal_store(Ct[c], st_off(K.C[c], pz + i0));
            }
        }
        if (q + 2 <= z1 + 1) fetch_main(q + 2);
        if (q + 3 <= z1 + 1) fetch_aux(q + 3);
        if (q + 1 <= z1) load_c(Cl, q + 1, q + 2);
        __syncthreads();
        // F^{k+1} at plane q
        if (bmain) {
            const int base = bslot + 2 * bly + W0X + 1;  // the same cell in the F^k window
            auto V = [&](int c, int dx, int dy, int dz) {
                const int s = dz < 0 ? am : (dz > 0 ? ap : ac);
                return A[s][c][base + dx + W0X * dy];
            };
            float out[6];
            next_iterate(V, bgx, Cu, out, Cn);
#pragma unroll
            for (int c = 0; c < 6; c++) Bs[bp][c][bslot] = out[c];
        }
        if (cop) {
            const int base = cslot + 2 * crow + W0X + 1;
            auto V = [&](int c, int dx, int dy, int dz) {
                const int s = dz < 0 ? am : (dz > 0 ? ap : ac);
                return A[s][c][base + dx + W0X * dy];
            };
            float out[6], cv[6];
            next_iterate(V, cgx, Cu, out, cv);
#pragma unroll
            for (int c = 0; c < 6; c++) Bs[bp][c][cslot] = out[c];
        } else if (cimg && face[cs]) {
#pragma unroll
            for (int c = 0; c < 6; c++)
                Bs[bp][c][cslot] = shear_lerp(XB[xbq][cs][c][crow], XB[xbq][cs][c][crow + 1], w1[cs]);
        }
        if (q + 1 <= z1) aux_iterate(Cu, xm, xc, xp, xbq ^ 1);  // opposite face, plane q + 1
        __syncthreads();
        // F^{k+2} at plane q - 1
        if (tmain && q - 1 >= z0) {
            const int base = bslot;
            auto V = [&](int c, int dx, int dy, int dz) {
                const int s = dz < 0 ? bm : (dz > 0 ? bp : bc);
                return Bs[s][c][base + dx + W1X * dy];
            };
            const float v0 = -K.sO * ((float)bgx - K.half_nx);
            const float vh = -K.sO * ((float)bgx + 0.5f - K.half_nx);
            float L[6];
            ksb_operator<true>(V, v0, vh, K.sO, L);
#pragma unroll
            for (int c = 0; c < 6; c++) Ores[c] = Ct[c] + h * L[c];
        }
#pragma unroll
        for (int c = 0; c < 6; c++) Ct[c] = FIRST ? Cn[c] : Cu[c];  // C at the tile cell, plane q
        int t = am;
        am = ac;
        ac = ap;
        ap = t;
        t = bm;
        bm = bc;
        bc = bp;
        bp = t;
        t = xm;
        xm = xc;
        xc = xp;
        xp = t;
        xbq ^= 1;
    };
    int q = z0 - 1;
    for (; q + 1 <= z1; q += 2) {
        plane(q, Ca, Cb);
        plane(q + 1, Cb, Ca);
    }
    if (q <= z1) plane(q, Ca, Cb);
    if (inside && z1 - 1 >= z0) {
        const uint32_t pz = plane_of(z1 - 1);
#pragma unroll
        for (int c = 0; c < 6; c++) __builtin_nontemporal_store(Ores[c], st_off(K.Fo[c], pz + i0));
    }
}

// End of a tolerance-mode step (one record per box): find the first sweep that met the
// tolerance, report the sweep count, latch kErrNoConverge if none did, and move that sweep's
// iterate into the set the step hands on when it sits in the other one.
__device__ __attribute__((always_inline)) inline void ksb_final_body(const KsbFin& F, int blk, int nblk, int)
{
    __shared__ int kstar;
    if (threadIdx.x == 0) {
        int k = F.K - 1;
        bool met = false;
        for (int j = 0; j < F.K && !met; j++)
            if (ksb_met(F.conv + 2 * j, F.tol)) {
                k = j;
                met = true;
            }
        kstar = k;
        if (blk == 0) {
            *F.sweeps = k + 1;
            if (!met) atomicOr(F.err, kErrNoConverge);
        }
    }
    __syncthreads();
    if (((F.K - 1 - kstar) & 1) == 0) return;
    const GridDev& G = F.G;
    const int64_t n = (int64_t)G.n[0] * G.n[1] * G.n[2];
    for (int64_t t = (int64_t)blk * kBlock + threadIdx.x; t < n; t += (int64_t)nblk * kBlock) {
        int x, y, z;
        cell_of(G, t, x, y, z);
        const int64_t i = gidx(G, x, y, z);
#pragma unroll
        for (int c = 0; c < 6; c++) F.dst[c][i] = F.src[c][i];
    }
}
PIC_BATCHED_KERNEL(ksb_final, KsbFin, kBlock)
#pragma clang fp contract(fast)

// ------------------------------------------------------------------ utilities
// interior of six components (B then E) times f[c % 3] (the expanding-frame conversion of the
// combined frame's field step)
// grid-stride over the cells (the batched launch gives every cell its own thread)
__device__ __attribute__((always_inline)) inline void scale_fields_body(const ScaleArgs& a, int blk, int nblk, int)
{
    const GridDev& G = a.G;
    const int64_t n = (int64_t)G.n[0] * G.n[1] * G.n[2];
    for (int64_t t = (int64_t)blk * kBlock + threadIdx.x; t < n; t += (int64_t)nblk * kBlock) {
        int x, y, z;
        cell_of(G, t, x, y, z);
        const int64_t i = gidx(G, x, y, z);
#pragma unroll
        for (int c = 0; c < 6; c++) a.F[c][i] *= a.f[c % 3];
    }
}
PIC_BATCHED_KERNEL(scale_fields, ScaleArgs, kBlock)

// grid-stride, 16-byte stores where the array is 16-byte aligned (the batched launch gives
// every word its own thread, so most of its threads find nothing to do)
__device__ __attribute__((always_inline)) inline void zero_body(const ZeroArgs& a, int blk, int nblk, int)
{
    const int64_t stride = (int64_t)nblk * kBlock, i = (int64_t)blk * kBlock + threadIdx.x;
    int64_t head = 0;
    if ((reinterpret_cast<uintptr_t>(a.p) & 15) == 0) {
        uint4* q = reinterpret_cast<uint4*>(a.p);
        const int64_t n4 = a.n >> 2;
        for (int64_t j = i; j < n4; j += stride) q[j] = make_uint4(0u, 0u, 0u, 0u);
        head = n4 << 2;
    }
    for (int64_t j = head + i; j < a.n; j += stride) a.p[j] = 0u;
}
PIC_BATCHED_KERNEL(zero, ZeroArgs, kBlock)

// interior <-> dense copies: dense index x + n0*(y + n1*z)
__global__ __launch_bounds__(kBlock) void interior_copy_kernel(GridDev G, float* guarded,
                                                               float* dense, int to_dense)
{
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (int64_t)G.n[0] * G.n[1] * G.n[2]) return;
    int x, y, z;
    cell_of(G, t, x, y, z);
    const int64_t i = gidx(G, x, y, z);
    if (to_dense)
        dense[t] = guarded[i];
    else
        guarded[i] = dense[t];
}

// FP64 block partial sums of squares of up to 6 interior component arrays
__global__ __launch_bounds__(kBlock) void field_energy_kernel(GridDev G, Comp6 A, double* part)
{
    __shared__ double sh[kBlock];
    const int c = blockIdx.y;
    double acc = 0.0;
    const int64_t ncell = (int64_t)G.n[0] * G.n[1] * G.n[2];
    for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < ncell;
         t += (int64_t)gridDim.x * kBlock) {
        int x, y, z;
        cell_of(G, t, x, y, z);
        const double v = A.p[c][gidx(G, x, y, z)];
        acc += v * v;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[c * gridDim.x + blockIdx.x] = sh[0];
}

// FP64 block partial sums of (gamma-1), u_x, u_y, u_z over the live particles
// sums over the particles that have not escaped (an escape marks the cell -1 until the next
// sort drops the particle)
__global__ __launch_bounds__(kBlock) void particle_sums_kernel(const int32_t* cell, const float* ux,
                                                               const float* uy, const float* uz,
                                                               const int32_t* n_live,
                                                               double* part)
{
    __shared__ double sh[kPartSums][kBlock];
    double a[kPartSums] = {};
    const int n = *n_live;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        if (cell[i] < 0) continue;
        const double x = ux[i], y = uy[i], z = uz[i];
        const double uu = x * x + y * y + z * z;
        const double g = sqrt(1.0 + uu);
        a[0] += uu / (g + 1.0);  // gamma - 1 without cancellation
        a[1] += x;
        a[2] += y;
        a[3] += z;
        a[4] += x * x / g;  // kinetic stress diagonal u_c^2 / gamma
        a[5] += y * y / g;
        a[6] += z * z / g;
    }
    for (int k = 0; k < kPartSums; k++) sh[k][threadIdx.x] = a[k];
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int k = 0; k < kPartSums; k++) sh[k][threadIdx.x] += sh[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < kPartSums; k++) part[k * gridDim.x + blockIdx.x] = sh[k][0];
}

// Energy distribution (Sec. 4.2) of the particles that have not escaped: slot = number of
// edges <= gamma - 1 (0: below the first edge, nbins + 1: at or above the last; non-finite
// energies go to the last slot).  Edges and the workgroup's counts sit in LDS; each workgroup
// adds its non-zero counts once.
__global__ __launch_bounds__(kBlock) void energy_hist_kernel(const int32_t* cell, const float* ux,
                                                             const float* uy, const float* uz,
                                                             const int32_t* n_live,
                                                             const double* edges, int nbins,
                                                             unsigned long long* counts)
{
    __shared__ double e[kHistMaxBins + 1];
    __shared__ uint32_t h[kHistMaxBins + 2];
    for (int b = threadIdx.x; b < nbins + 2; b += kBlock) h[b] = 0u;
    for (int b = threadIdx.x; b <= nbins; b += kBlock) e[b] = edges[b];
    __syncthreads();
    const int n = *n_live;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        if (cell[i] < 0) continue;
        const double x = ux[i], y = uy[i], z = uz[i];
        const double uu = x * x + y * y + z * z;  // FP32 inputs: the products are exact
        const double k = uu / (sqrt(1.0 + uu) + 1.0);
        int lo = 0, hi = nbins + 1;  // edges[0..lo) <= k, edges[hi..] > k
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (e[mid] <= k)
                lo = mid + 1;
            else
                hi = mid;
        }
        atomicAdd(&h[k == k ? lo : nbins + 1], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nbins + 2; b += kBlock)
        if (h[b]) atomicAdd(&counts[b], (unsigned long long)h[b]);
}

// fixed-order final sum of nrow rows of ncol partials (one thread per row)
__global__ void sum_rows_kernel(const double* part, int nrow, int ncol, double* out)
{
    const int r = threadIdx.x;
    if (r >= nrow) return;
    double s = 0.0;
    for (int k = 0; k < ncol; k++) s += part[r * ncol + k];
    out[r] = s;
}

// ------------------------------------------------------------------ host launchers
static inline unsigned nblocks(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }
// grid of the grid-stride cell kernels (the shear fold, the Yee updates): 16 blocks per CU,
// each thread taking a few cells, measured faster than one thread per cell (fold at 256^3:
// 0.18 against 0.22 ms)
constexpr unsigned kStrideBlocks = 4096;

hipError_t fill_guards(const GridDev& G, float* const* comps, int ncomp, int shear, double dys,
                       hipStream_t st)
{
    Comp6 A{};
    for (int c = 0; c < ncomp; c++) A.p[c] = comps[c];
    const double fl = floor(dys);
    const int di = (int)fl;
    const float w = (float)(dys - fl);
    const int NYg = G.n[1] + 2 * G.g[1], NZg = G.n[2] + 2 * G.g[2];
    fill_guards_kernel<<<dim3(nblocks((int64_t)2 * G.g[0] * NYg * NZg), ncomp), kBlock, 0, st>>>(
        FillArgs{G, A, 0, shear, di, w});
    fill_guards_kernel<<<dim3(nblocks((int64_t)G.n[0] * 2 * G.g[1] * NZg), ncomp), kBlock, 0, st>>>(
        FillArgs{G, A, 1, shear, di, w});
    if (G.g[2] > 0)
        fill_guards_kernel<<<dim3(nblocks((int64_t)G.n[0] * G.n[1] * 2 * G.g[2]), ncomp), kBlock, 0,
                             st>>>(FillArgs{G, A, 2, shear, di, w});
    return hipGetLastError();
}

// Fold the deposited current.  For the shearing box tmp receives the transported current and
// the fold writes every interior cell of J.
hipError_t fold_current(const GridDev& G, float* const* J, float* const* out, int shear,
                        double sO, double dt, double dys_half, hipStream_t st)
{
    Comp3 Jc{{J[0], J[1], J[2]}};
    const int NXg = G.n[0] + 2 * G.g[0], NYg = G.n[1] + 2 * G.g[1];
    if (G.g[2] > 0) {
        const int nl = G.n[2] < 2 * G.g[2] ? G.n[2] : 2 * G.g[2];
        fold_periodic_kernel<<<dim3(nblocks((int64_t)NXg * NYg * nl), 3), kBlock, 0, st>>>(
            FoldPArgs{G, Jc, 2});
    }
    {
        const int nl = G.n[1] < 2 * G.g[1] ? G.n[1] : 2 * G.g[1];
        fold_periodic_kernel<<<dim3(nblocks((int64_t)NXg * nl * G.n[2]), 3), kBlock, 0, st>>>(
            FoldPArgs{G, Jc, 1});
    }
    const double fl = floor(dys_half);
    const int di = (int)fl;
    const float w = (float)(dys_half - fl);
    if (shear) {
        Comp3 Oc{{out[0], out[1], out[2]}};
        const unsigned nb = std::min(nblocks((int64_t)G.n[0] * G.n[1] * G.n[2]), kStrideBlocks);
        shear_fold_kernel<<<dim3(nb, 3), kBlock, 0, st>>>(
            ShearFoldArgs{G, Jc, Oc, (float)(sO * dt / 2.0), 0.5f * G.n[0], di, w});
    } else {
        const int nl = G.n[0] < 2 * G.g[0] ? G.n[0] : 2 * G.g[0];
        fold_x_kernel<<<dim3(nblocks((int64_t)nl * G.n[1] * G.n[2]), 3), kBlock, 0, st>>>(
            FoldXArgs{G, Jc, Jc, 0, 0, 0, 0.f});
    }
    return hipGetLastError();
}

hipError_t yee_b(const MaxwellDev& M, hipStream_t st)
{
    yee_b_kernel<<<std::min(nblocks((int64_t)M.G.n[0] * M.G.n[1] * M.G.n[2]), kStrideBlocks), kBlock, 0, st>>>(M);
    return hipGetLastError();
}
hipError_t yee_e(const MaxwellDev& M, hipStream_t st)
{
    yee_e_kernel<<<std::min(nblocks((int64_t)M.G.n[0] * M.G.n[1] * M.G.n[2]), kStrideBlocks), kBlock, 0, st>>>(M);
    return hipGetLastError();
}
bool ksb_staged(const GridDev& G) { return G.dim == 3 && G.n[0] % KX == 0; }
bool ksb_pass_fits(const GridDev& G)
{
    return G.dim == 3 && G.n[0] % kPassX == 0 && 4 * (int64_t)G.sz * G.n[2] < (int64_t(1) << 32);
}

hipError_t ksb_sweep(const KsbDev& K, bool first, hipStream_t st)
{
    if (ksb_staged(K.G)) {
        const unsigned grid = (unsigned)((K.G.n[0] / KX) * ((K.G.n[1] + KY - 1) / KY) *
                                         ((K.G.n[2] + KZ - 1) / KZ));
        if (first)
            ksb_sweep3_kernel<true><<<grid, KX * KY, 0, st>>>(K);
        else
            ksb_sweep3_kernel<false><<<grid, KX * KY, 0, st>>>(K);
    } else {
        const unsigned nb = nblocks((int64_t)K.G.n[0] * K.G.n[1] * K.G.n[2]);
        if (first)
            ksb_first_kernel<<<nb, kBlock, 0, st>>>(K);
        else
            ksb_next_kernel<<<nb, kBlock, 0, st>>>(K);
    }
    return hipGetLastError();
}
hipError_t ksb_sweep_unstaged(const KsbDev& K, bool first, hipStream_t st)
{
    const unsigned nb = nblocks((int64_t)K.G.n[0] * K.G.n[1] * K.G.n[2]);
    if (first)
        ksb_first_kernel<<<nb, kBlock, 0, st>>>(K);
    else
        ksb_next_kernel<<<nb, kBlock, 0, st>>>(K);
    return hipGetLastError();
}
hipError_t ksb_pass(const KsbDev& K, bool first, hipStream_t st)
{
    if (!ksb_pass_fits(K.G) || K.conv) return hipErrorInvalidValue;
    using T = PassTile<kPassX>;
    const unsigned grid = (unsigned)((K.G.n[0] / T::PX) * ((K.G.n[1] + T::PY - 1) / T::PY) *
                                     ((K.G.n[2] + T::PZ - 1) / T::PZ));
    if (first)
        ksb_pass3_kernel<kPassX, true><<<grid, T::PN, 0, st>>>(K);
    else
        ksb_pass3_kernel<kPassX, false><<<grid, T::PN, 0, st>>>(K);
    return hipGetLastError();
}
hipError_t scale_fields(const GridDev& G, float* const* F, const float f[3], hipStream_t st)
{
    ScaleArgs a{};
    a.G = G;
    for (int c = 0; c < 6; c++) a.F[c] = F[c];
    for (int c = 0; c < 3; c++) a.f[c] = f[c];
    scale_fields_kernel<<<std::min(nblocks((int64_t)G.n[0] * G.n[1] * G.n[2]), kStrideBlocks), kBlock, 0, st>>>(a);
    return hipGetLastError();
}
hipError_t ksb_finalize(const KsbFin& F, hipStream_t st)
{
    ksb_final_kernel<<<kKsbFinBlocks, kBlock, 0, st>>>(F);
    return hipGetLastError();
}
hipError_t grid_batch(GridBatchKind k, const void* table, UnitMap m, int blocks, int ydim,
                      hipStream_t st)
{
    if (blocks <= 0) return hipSuccess;
    const dim3 grid((unsigned)blocks, (unsigned)ydim);
    switch (k) {
    case kBatchZero: zero_batch<<<grid, kBlock, 0, st>>>(static_cast<const ZeroArgs*>(table), m); break;
    case kBatchFill:
        fill_guards_batch<<<grid, kBlock, 0, st>>>(static_cast<const FillArgs*>(table), m);
        break;
    case kBatchFoldP:
        fold_periodic_batch<<<grid, kBlock, 0, st>>>(static_cast<const FoldPArgs*>(table), m);
        break;
    case kBatchShearFold:
        shear_fold_batch<<<grid, kBlock, 0, st>>>(static_cast<const ShearFoldArgs*>(table), m);
        break;
    case kBatchFoldX: fold_x_batch<<<grid, kBlock, 0, st>>>(static_cast<const FoldXArgs*>(table), m); break;
    case kBatchYeeB: yee_b_batch<<<grid, kBlock, 0, st>>>(static_cast<const MaxwellDev*>(table), m); break;
    case kBatchYeeE: yee_e_batch<<<grid, kBlock, 0, st>>>(static_cast<const MaxwellDev*>(table), m); break;
    case kBatchKsbFirst:
        ksb_first_batch<<<grid, kBlock, 0, st>>>(static_cast<const KsbDev*>(table), m);
        break;
    case kBatchKsbNext: ksb_next_batch<<<grid, kBlock, 0, st>>>(static_cast<const KsbDev*>(table), m); break;
    case kBatchKsbFinal: ksb_final_batch<<<grid, kBlock, 0, st>>>(static_cast<const KsbFin*>(table), m); break;
    case kBatchScale: scale_fields_batch<<<grid, kBlock, 0, st>>>(static_cast<const ScaleArgs*>(table), m); break;
    }
    return hipGetLastError();
}

unsigned grid_blocks(int64_t items) { return nblocks(items); }

hipError_t zero_floats(float* p, int64_t n, hipStream_t st)
{
    if (n > 0)
        zero_kernel<<<std::min(nblocks((n + 3) / 4), kStrideBlocks), kBlock, 0, st>>>(
            ZeroArgs{reinterpret_cast<uint32_t*>(p), n});
    return hipGetLastError();
}
hipError_t interior_copy(const GridDev& G, float* guarded, float* dense, int to_dense, hipStream_t st)
{
    interior_copy_kernel<<<nblocks((int64_t)G.n[0] * G.n[1] * G.n[2]), kBlock, 0, st>>>(G, guarded,
                                                                                      dense, to_dense);
    return hipGetLastError();
}
hipError_t field_energy(const GridDev& G, float* const* comps, int ncomp, double* part, int nblk,
                        double* out, hipStream_t st)
{
    Comp6 A{};
    for (int c = 0; c < ncomp; c++) A.p[c] = comps[c];
    field_energy_kernel<<<dim3(nblk, ncomp), kBlock, 0, st>>>(G, A, part);
    sum_rows_kernel<<<1, 64, 0, st>>>(part, ncomp, nblk, out);
    return hipGetLastError();
}
hipError_t particle_sums(const int32_t* cell, const float* ux, const float* uy, const float* uz,
                         const int32_t* n_live, double* part, int nblk, double* out, hipStream_t st)
{
    particle_sums_kernel<<<nblk, kBlock, 0, st>>>(cell, ux, uy, uz, n_live, part);
    sum_rows_kernel<<<1, 64, 0, st>>>(part, kPartSums, nblk, out);
    return hipGetLastError();
}
hipError_t energy_histogram(const int32_t* cell, const float* ux, const float* uy, const float* uz,
                            const int32_t* n_live, const double* edges, int nbins,
                            unsigned long long* counts, int nblk, hipStream_t st)
{
    zero_kernel<<<nblocks(2 * (nbins + 2)), kBlock, 0, st>>>(
        ZeroArgs{reinterpret_cast<uint32_t*>(counts), (int64_t)2 * (nbins + 2)});
    energy_hist_kernel<<<nblk, kBlock, 0, st>>>(cell, ux, uy, uz, n_live, edges, nbins, counts);
    return hipGetLastError();
}

}  // namespace pic
