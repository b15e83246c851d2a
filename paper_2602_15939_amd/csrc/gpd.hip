// gpd.hip — the particle hot path on gfx950: field gather from the Yee grid, the frame's
// Boris-like push, position update with the boundary conditions, leaky-box escape and the
// charge-conserving (Esirkepov) current deposit, fused in one kernel per tile.
//
// One workgroup owns one tile: it stages E and B of the tile plus the guard layers the gather
// reaches in LDS (one region per Yee component, sized for that component's lattice),
// accumulates the tile's current (plus the deposit halo) in LDS as 64-bit fixed point, and
// flushes it once to HBM with float atomics (only the halo overlaps a neighbour tile).
// Particles are read through the sort permutation and written in sorted slot order, so the
// tile sort's scatter is fused into this pass.  A particle found outside its tile (only
// possible without a sort since the last push) takes the global-memory path.
#include "pic_internal.h"

namespace pic {

// ------------------------------------------------------------------ small vector helpers
struct f3 {
    float x, y, z;
};
__device__ inline f3 mk(float a, float b, float c) { return f3{a, b, c}; }
__device__ inline f3 operator+(f3 a, f3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ inline f3 operator*(float s, f3 a) { return mk(s * a.x, s * a.y, s * a.z); }
__device__ inline float dot(f3 a, f3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline f3 cross(f3 a, f3 b)
{
    return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}

// Hardware reciprocal and square root (v_rcp_f32, v_sqrt_f32: about 1 ulp), used instead of
// the correctly rounded division and square-root sequences.
__device__ inline float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
// v_rsq_f32 for arguments >= 1 (Lorentz factors): no denormal rescaling needed
__device__ inline float rsq1(float x) { return __builtin_amdgcn_rsqf(x); }

// Particle arrays are indexed with 32-bit byte offsets (capacity below 2^30 per species), so
// the loads and stores take a scalar base and one shared vector offset.
template <class T>
__device__ inline T ld_at(const T* __restrict__ base, uint32_t i)
{
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) +
                                       (size_t)(i * (uint32_t)sizeof(T)));
}
template <class T>
__device__ inline void st_at(T* __restrict__ base, uint32_t i, T v)
{
    *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + (size_t)(i * (uint32_t)sizeof(T))) = v;
}

// ------------------------------------------------------------------ interpolation
// Linear (CIC) interpolation of one component on its own staggered lattice (base index and
// weights per axis), from an array with element strides (1, sy, sz).
template <int DIM>
__device__ inline float interp(const float* __restrict__ F, int bx, int by, int bz, float wx,
                               float wy, float wz, int sy, int sz)
{
    const float* p = F + bx + sy * by + (DIM == 3 ? sz * bz : 0);
    float a = p[0] + wx * (p[1] - p[0]);
    float b = p[sy] + wx * (p[sy + 1] - p[sy]);
    float r = a + wy * (b - a);
    if (DIM == 3) {
        const float* q = p + sz;
        float c = q[0] + wx * (q[1] - q[0]);
        float d = q[sy] + wx * (q[sy + 1] - q[sy]);
        float r2 = c + wy * (d - c);
        r = r + wz * (r2 - r);
    }
    return r;
}

// Per axis: the integer lattice uses (cell, offset); the half-shifted lattice uses
// (cell-1, offset+1/2) below the cell centre and (cell, offset-1/2) above it.
struct AxisW {
    int b0, bh;
    float w0, wh;
};
__device__ inline AxisW axis_weights(int c, float o)
{
    AxisW a;
    const bool lo = o < 0.5f;
    a.b0 = c;
    a.w0 = o;
    a.bh = lo ? c - 1 : c;
    a.wh = lo ? o + 0.5f : o - 0.5f;
    return a;
}

// Gather the six Yee components at a particle.  Fields are arrays 0..2 = E, 3..5 = B.
template <int DIM, class FieldAt>
__device__ inline void gather(FieldAt fa, int sy, int sz, int cx, int cy, int cz, float ox,
                              float oy, float oz, f3& E, f3& B)
{
    const AxisW X = axis_weights(cx, ox), Y = axis_weights(cy, oy);
    AxisW Z = axis_weights(cz, oz);
    if (DIM == 2) Z = AxisW{0, 0, 0.f, 0.f};
    E.x = interp<DIM>(fa(0), X.bh, Y.b0, Z.b0, X.wh, Y.w0, Z.w0, sy, sz);
    E.y = interp<DIM>(fa(1), X.b0, Y.bh, Z.b0, X.w0, Y.wh, Z.w0, sy, sz);
    E.z = interp<DIM>(fa(2), X.b0, Y.b0, Z.bh, X.w0, Y.w0, Z.wh, sy, sz);
    B.x = interp<DIM>(fa(3), X.b0, Y.bh, Z.bh, X.w0, Y.wh, Z.wh, sy, sz);
    B.y = interp<DIM>(fa(4), X.bh, Y.b0, Z.bh, X.wh, Y.w0, Z.wh, sy, sz);
    B.z = interp<DIM>(fa(5), X.bh, Y.bh, Z.b0, X.wh, Y.wh, Z.w0, sy, sz);
}

// ------------------------------------------------------------------ pushers
// Standard Boris (the alpha = 0 and Lambda = 0 limits of the operators of Secs. 2.2, 3.2).
__device__ inline f3 push_boris(f3 u, f3 E, f3 B, float qm_hdt)
{
    const f3 eps = qm_hdt * E;
    const f3 um = u + eps;
    const float ig = rsq1(1.f + dot(um, um));
    const f3 t = (qm_hdt * ig) * B;
    const float d = 2.f * rcp(1.f + dot(t, t));
    const f3 c1 = cross(um, t);
    const f3 c2 = cross(c1, t);
    return um + d * (c1 + c2) + eps;
}

// Shearing-box push (Sec. 2.2, eq. OAu_disc): closed form
//   u+ = B(u-) + R(S u-) + R(S w)/(1-g),  w = B(u-) + R(S u-),  g = S_2 . R(e_y),
// with S u = e_y (s2 . u); R(e_y) written out.  gamma-bar from the printed first-order
// approximation refined by one fixed-point step of g^2 = 1 + A + K/g (the step contracts by
// about |K|/(2 g^3), so the approximation's error, at most ~4e-7, drops below FP32 rounding).
__device__ inline f3 push_shear(f3 u, f3 E, f3 B, float qm_hdt, float alpha1, float alpha2,
                                float om_dt)
{
    const f3 eps = qm_hdt * E;
    const f3 um = u + eps;
    const float uu = dot(um, um);
    const float ue = dot(um, eps);
    const float A = uu + 2.f * alpha1 * um.x * um.y;
    const float K = 2.f * alpha2 * ue * um.y;
    const float g0 = fsqrt(1.f + uu);
    float g = g0 + (alpha1 * um.x * um.y * g0 + alpha2 * ue * um.y) * rcp(1.f + uu);
    g = fsqrt(1.f + A + K * rcp(g));
    const float ig = rcp(g);
    f3 t = (qm_hdt * ig) * B;
    t.z += om_dt;
    const f3 et = ig * eps;
    const f3 s2 = mk(alpha1 + alpha2 * et.x, alpha2 * et.y, alpha2 * et.z);
    const float d = rcp(1.f + dot(t, t));
    const f3 c1 = cross(um, t);
    const f3 c2 = cross(c1, t);
    const f3 Bu = um + (2.f * d) * (c1 + c2);
    const f3 Rey = mk(d * (t.z + t.x * t.y), 1.f - d * (t.x * t.x + t.z * t.z), d * (t.y * t.z - t.x));
    const float gg = dot(s2, Rey);
    const f3 w = Bu + dot(s2, um) * Rey;
    const f3 up = w + (dot(s2, w) * rcp(1.f - gg)) * Rey;
    return up + eps;
}

// Expanding-box push (Sec. 3.2, eq. EBu_disc) with the printed modified Boris operator
//   B^(L)(v) = L~ v + ((1+L~) v x t~ + ((1+L~) v x t~) x t~)/(1 + t~^2),
// gamma-bar = sqrt(1 + ((1+Lambda) u-)^2), t~ = tau/(1-Lambda).
__device__ inline f3 push_expand(f3 u, f3 E, f3 B, float qm_hdt, const float lam1p[3],
                                 const float ltil[3], const float tfac[3])
{
    const f3 eps = qm_hdt * E;
    const f3 um = u + eps;
    const f3 lu = mk(lam1p[0] * um.x, lam1p[1] * um.y, lam1p[2] * um.z);
    const float ig = rsq1(1.f + dot(lu, lu));
    const float s = qm_hdt * ig;
    const f3 t = mk(s * tfac[0] * B.x, s * tfac[1] * B.y, s * tfac[2] * B.z);
    const f3 w = mk((1.f + ltil[0]) * um.x, (1.f + ltil[1]) * um.y, (1.f + ltil[2]) * um.z);
    const float d = rcp(1.f + dot(t, t));
    const f3 c1 = cross(w, t);
    const f3 c2 = cross(c1, t);
    const f3 up = mk(ltil[0] * um.x, ltil[1] * um.y, ltil[2] * um.z) + d * (c1 + c2);
    return up + eps;
}

// Combined shearing and expanding frame (the extension named in the conclusion, Sec. 5;
// reading): (1 - Lambda) u+ - u+ x tau~ - S u+ = (1 + Lambda) u- + u- x tau~ + S u-, i.e.
// eq. OAu_disc with the diagonal Lambda of eq. EBu_disc.  A u = (1 - Lambda) u - u x tau~ is
// inverted as the expanding push does, A^-1 r = R_t((1 - Lambda)^-1 r), t = (1 - Lambda)^-1
// tau~, so A^-1((1 + Lambda) v + v x tau~) is the printed B^(Lambda)(v); the rank-1 S is added
// by the Sherman-Morrison formula, as the shearing push adds it to R:
//   w = B^(Lambda)(u-) + (s2.u-) A^-1 e_y,  u+ = w + (s2.w) A^-1 e_y / (1 - s2.A^-1 e_y).
// gamma-bar solves g^2 = 1 + ((1+Lambda)u-)^2 + 2 alpha1 u-_x u-_y + 2 alpha2 (u-.eps) u-_y / g:
// the shearing push's first-order approximation (with (1+Lambda) u- in place of u-) and one
// fixed-point refinement.  Lambda = 0 is the shearing push, alpha = Omega0 = 0 the expanding.
__device__ inline f3 push_shear_expand(f3 u, f3 E, f3 B, float qm_hdt, float alpha1, float alpha2,
                                       float om_dt, const float lam1p[3], const float ltil[3],
                                       const float tfac[3])
{
    const f3 eps = qm_hdt * E;
    const f3 um = u + eps;
    const f3 lu = mk(lam1p[0] * um.x, lam1p[1] * um.y, lam1p[2] * um.z);
    const float ll = dot(lu, lu);
    const float ue = dot(um, eps);
    const float A = ll + 2.f * alpha1 * um.x * um.y;
    const float K = 2.f * alpha2 * ue * um.y;
    const float g0 = fsqrt(1.f + ll);
    float g = g0 + (alpha1 * um.x * um.y * g0 + alpha2 * ue * um.y) * rcp(1.f + ll);
    g = fsqrt(1.f + A + K * rcp(g));
    const float ig = rcp(g);
    f3 tt = (qm_hdt * ig) * B;
    tt.z += om_dt;
    const f3 t = mk(tfac[0] * tt.x, tfac[1] * tt.y, tfac[2] * tt.z);
    const f3 et = ig * eps;
    const f3 s2 = mk(alpha1 + alpha2 * et.x, alpha2 * et.y, alpha2 * et.z);
    const float d = rcp(1.f + dot(t, t));
    const f3 v = mk((1.f + ltil[0]) * um.x, (1.f + ltil[1]) * um.y, (1.f + ltil[2]) * um.z);
    const f3 c1 = cross(v, t);
    const f3 c2 = cross(c1, t);
    const f3 Bu = mk(ltil[0] * um.x, ltil[1] * um.y, ltil[2] * um.z) + d * (c1 + c2);
    // A^-1 e_y = R_t(e_y) / (1 - Lambda_y), R_t(e_y) written out
    const f3 Ae = tfac[1] * mk(d * (t.z + t.x * t.y), 1.f - d * (t.x * t.x + t.z * t.z), d * (t.y * t.z - t.x));
    const float gg = dot(s2, Ae);
    const f3 w = Bu + dot(s2, um) * Ae;
    const f3 up = w + (dot(s2, w) * rcp(1.f - gg)) * Ae;
    return up + eps;
}

// ------------------------------------------------------------------ positions
// In-cell offset renormalisation after s = off + delta (|delta| < 1), in FP32:
// s >= 1 -> (+1, s-1) exact; s < 0 -> t = s+1, (-1, t) if t < 1 else (0, 0).  Written with
// selects only (no divergent branches).
__device__ inline float renorm(float s, int& dc)
{
    const float sm = __fsub_rn(s, 1.f), sp = __fadd_rn(s, 1.f);
    const bool ge = s >= 1.f, lt = s < 0.f, lt_ok = lt && sp < 1.f;
    dc = ge ? 1 : (lt_ok ? -1 : 0);
    return ge ? sm : (lt ? (lt_ok ? sp : 0.f) : s);
}

// ------------------------------------------------------------------ Esirkepov deposit
// CIC shape on the 3 nodes nearest-1..nearest+1 of one axis, xi = position - nearest node.
struct Shape3 {
    float s0[3], ds[3];
    float lo, hi;  // min and max of the old and new position relative to the nearest node
};
__device__ inline Shape3 shape3(float xi0, float xi1)
{
    Shape3 S;
    S.lo = fminf(xi0, xi1);
    S.hi = fmaxf(xi0, xi1);
    const float a0 = fmaxf(0.f, -xi0), b0 = 1.f - fabsf(xi0), c0 = fmaxf(0.f, xi0);
    const float a1 = fmaxf(0.f, -xi1), b1 = 1.f - fabsf(xi1), c1 = fmaxf(0.f, xi1);
    S.s0[0] = a0;
    S.s0[1] = b0;
    S.s0[2] = c0;
    S.ds[0] = a1 - a0;
    S.ds[1] = b1 - b0;
    S.ds[2] = c1 - c0;
    return S;
}

// Esirkepov decomposition of the density change into currents (CIC):
//   J_x on the two edges around the nearest node: -q/dt DS_x[-1] P and +q/dt DS_x[+1] P,
//   P = S0_y (S0_z + DS_z/2) + DS_y (S0_z/2 + DS_z/3) (cyclic for y and z);
//   2D: P = S0_y + DS_y/2, and J_z = q dz/dt (S0_x (S0_y + DS_y/2) + DS_x (S0_y/2 + DS_y/3)).
// Acc::add(c, x, y, z, v, on) accumulates v into component c at (edge/node) index (x, y, z)
// relative to the nearest node minus one.  `on` is false only where v is exactly zero: an outer
// node that neither the old nor the new shape touches, or an edge whose DS factor is zero.  A
// particle that stays on one side of its nearest node in every axis has 12 (3D) / 10 (2D)
// non-zero terms out of 54 / 21, and skipping the rest leaves the integer sums unchanged.
// The lower outer node is touched by the old or the new shape exactly when one of the two
// positions lies below the nearest node (S0 or S1 of that node non-zero), the upper one when one
// lies above.  An outer edge carries current only if its outer node is touched (its DS can still
// be zero, for an unmoved coordinate: the term then adds an exact zero).
struct Use3 {
    bool n0, n2;  // outer nodes touched by the old or the new shape
    bool e0, e2;  // the two outer edges may carry current
};
__device__ inline Use3 use3(const Shape3& S)
{
    const bool n0 = S.lo < 0.f, n2 = S.hi > 0.f;
    return Use3{n0, n2, n0, n2};
}
__device__ inline bool used(const Use3& U, int b) { return b == 0 ? U.n0 : (b == 2 ? U.n2 : true); }

template <int DIM, class Acc>
__device__ inline void esirkepov(Acc& acc, const Shape3& X, const Shape3& Y, const Shape3& Z,
                                 float q_dt, float dz)
{
    const Use3 UX = use3(X), UY = use3(Y);
    if (DIM == 3) {
        const Use3 UZ = use3(Z);
        // transverse factors with the charge factor q/dt folded in, so that every term is one
        // product of a DS value and a factor
        const float qh = 0.5f * q_dt, qt = (1.f / 3.f) * q_dt;
        float z1[3], z2[3], y1[3], y2[3];
#pragma unroll
        for (int c = 0; c < 3; c++) {
            z1[c] = q_dt * Z.s0[c] + qh * Z.ds[c];
            z2[c] = qh * Z.s0[c] + qt * Z.ds[c];
            y1[c] = q_dt * Y.s0[c] + qh * Y.ds[c];
            y2[c] = qh * Y.s0[c] + qt * Y.ds[c];
        }
#pragma unroll
        for (int b = 0; b < 3; b++)
#pragma unroll
            for (int c = 0; c < 3; c++) {
                const bool yz = used(UY, b) && used(UZ, c);
                const float Pyz = Y.s0[b] * z1[c] + Y.ds[b] * z2[c];
                acc.add(0, 0, b, c, -X.ds[0] * Pyz, UX.e0 && yz);
                acc.add(0, 1, b, c, X.ds[2] * Pyz, UX.e2 && yz);
                const bool xz = used(UX, b) && used(UZ, c);
                const float Pxz = X.s0[b] * z1[c] + X.ds[b] * z2[c];
                acc.add(1, b, 0, c, -Y.ds[0] * Pxz, UY.e0 && xz);
                acc.add(1, b, 1, c, Y.ds[2] * Pxz, UY.e2 && xz);
                const bool xy = used(UX, b) && used(UY, c);
                const float Pxy = X.s0[b] * y1[c] + X.ds[b] * y2[c];
                acc.add(2, b, c, 0, -Z.ds[0] * Pxy, UZ.e0 && xy);
                acc.add(2, b, c, 1, Z.ds[2] * Pxy, UZ.e2 && xy);
            }
    } else {
        const float xl = -q_dt * X.ds[0], xh = q_dt * X.ds[2];
        const float yl = -q_dt * Y.ds[0], yh = q_dt * Y.ds[2];
        const float jz = q_dt * dz;
#pragma unroll
        for (int b = 0; b < 3; b++) {
            const float Py = Y.s0[b] + 0.5f * Y.ds[b];
            acc.add(0, 0, b, 0, xl * Py, UX.e0 && used(UY, b));
            acc.add(0, 1, b, 0, xh * Py, UX.e2 && used(UY, b));
            const float Px = X.s0[b] + 0.5f * X.ds[b];
            acc.add(1, b, 0, 0, yl * Px, UY.e0 && used(UX, b));
            acc.add(1, b, 1, 0, yh * Px, UY.e2 && used(UX, b));
        }
#pragma unroll
        for (int a = 0; a < 3; a++) {
#pragma unroll
            for (int b = 0; b < 3; b++) {
                const float W = X.s0[a] * (Y.s0[b] + 0.5f * Y.ds[b]) +
                                X.ds[a] * (0.5f * Y.s0[b] + (1.f / 3.f) * Y.ds[b]);
                acc.add(2, a, b, 0, jz * W, used(UX, a) && used(UY, b));
            }
        }
    }
}

// ------------------------------------------------------------------ tile regions in LDS
// Field component f (0..2 = Ex, Ey, Ez; 3..5 = Bx, By, Bz) lies on the half-shifted lattice
// along the axes of its Yee offset: Ex x, Ey y, Ez z, Bx y and z, By x and z, Bz x and y.
__host__ __device__ constexpr bool yee_half(int f, int a) { return f < 3 ? f == a : f - 3 != a; }

template <int DIM, int TX, int TY, int TZ>
struct Geo {
    static constexpr int T(int a) { return a == 0 ? TX : (a == 1 ? TY : TZ); }
    // Staged field component f: along a half-lattice axis the values at global indices
    // t0-1 .. t0+T (T+2), along an integer axis t0 .. t0+T (T+1): what CIC needs for a
    // particle in the tile.
    static constexpr int fdim(int f, int a)
    {
        return (DIM == 2 && a == 2) ? 1 : T(a) + (yee_half(f, a) ? 2 : 1);
    }
    static constexpr int fsize(int f) { return fdim(f, 0) * fdim(f, 1) * fdim(f, 2); }
    static constexpr int foff(int f) { return f == 0 ? 0 : foff(f - 1) + fsize(f - 1); }
    // Current component c, origin at global index t0-1 on every axis: along its own axis the
    // edges t0-1 .. t0+T (T+2), across it the nodes t0-1 .. t0+T+1 (T+3); the deposit of a
    // particle of the tile stays inside.  2D: J_z has nodes along x and y.
    static constexpr int jdim(int c, int a)
    {
        return (DIM == 2 && a == 2) ? 1 : T(a) + (a == c ? 2 : 3);
    }
    static constexpr int jsize(int c) { return jdim(c, 0) * jdim(c, 1) * jdim(c, 2); }
    static constexpr int joff(int c) { return c == 0 ? 0 : joff(c - 1) + jsize(c - 1); }
    static constexpr int JTOT = joff(2) + jsize(2);
    static constexpr int FTOT = foff(5) + fsize(5);
    static constexpr int FBYTES = (4 * FTOT + 15) & ~15;   // E, B first, then J (8-byte words)
    static constexpr int LDS_BYTES = FBYTES + 8 * JTOT;
};

// LDS accumulator: one region per current component (Geo::jdim).  The tile current is summed in
// 64-bit fixed point: a contribution arrives pre-scaled so that the largest possible single
// contribution is 2^30 units, is truncated to int32 and added with ds_add_u64 (integer LDS
// atomics cost a few cycles per wave instruction, while FP32 LDS atomics are serialised per
// lane).  Integer sums are exact and independent of the order.
template <class G>
struct LdsAcc {
    unsigned long long* J;
    int base[3];  // per component: region index of (nearest node - 1) on every axis
    __device__ inline void add(int c, int x, int y, int z, float v, bool on)
    {
        const long long q = (long long)(int)v;  // v_cvt_i32_f32: truncates, saturates
        if (on)
            atomicAdd(&J[G::joff(c) + base[c] + x + G::jdim(c, 0) * (y + G::jdim(c, 1) * z)],
                      (unsigned long long)q);
    }
};

// Global accumulator on the guarded current arrays (slow path).
struct GlobalAcc {
    float* const* J;
    int64_t base;
    int sy, sz;
    __device__ inline void add(int c, int x, int y, int z, float v, bool)
    {
        if (v != 0.f) unsafeAtomicAdd(&J[c][base + x + (int64_t)sy * y + (int64_t)sz * z], v);
    }
};

// CIC interpolation of staged component F: (ia, ib, ic) is the region index of the lower
// corner, (wa, wb, wc) the weights of the upper corner.  The eight corners are fixed offsets
// from one LDS address.
template <class G, int DIM, int F>
__device__ inline float interp_lds(const float* __restrict__ Fl, int ia, int ib, int ic, float wa,
                                   float wb, float wc)
{
    constexpr unsigned X = G::fdim(F, 0), XY = X * G::fdim(F, 1);
    // 24-bit multiply-adds (full rate); the index is non-negative and below 2^16
    const unsigned idx = (unsigned)G::foff(F) + (unsigned)ia + __umul24((unsigned)ib, X) +
                         (DIM == 3 ? __umul24((unsigned)ic, XY) : 0u);
    unsigned ad = idx;
    // opaque to constant reassociation: the corner offsets then fold into the ds_read2
    // immediates of one address register
    asm("" : "+v"(ad));
    const float* p = Fl + ad;
    const float a = p[0] + wa * (p[1] - p[0]);
    const float b = p[X] + wa * (p[X + 1] - p[X]);
    float r = a + wb * (b - a);
    if (DIM == 3) {
        const float* q = p + XY;
        const float c = q[0] + wa * (q[1] - q[0]);
        const float d = q[X] + wa * (q[X + 1] - q[X]);
        const float r2 = c + wb * (d - c);
        r = r + wc * (r2 - r);
    }
    return r;
}

// Gather from the staged tile: (rx, ry, rz) = cell - tile origin.  On a half-shifted axis the
// lower node is the one at cell - 1/2 below the cell centre and cell + 1/2 above it.
template <class G, int DIM>
__device__ inline void gather_lds(const float* __restrict__ Fl, int rx, int ry, int rz, float ox,
                                  float oy, float oz, f3& E, f3& B)
{
    const bool lx = ox < 0.5f, ly = oy < 0.5f, lz = oz < 0.5f;
    const float hx = ox + (lx ? 0.5f : -0.5f), hy = oy + (ly ? 0.5f : -0.5f);
    const float hz = oz + (lz ? 0.5f : -0.5f);
    const int ix = rx + (lx ? 0 : 1), iy = ry + (ly ? 0 : 1), iz = rz + (lz ? 0 : 1);
    E.x = interp_lds<G, DIM, 0>(Fl, ix, ry, rz, hx, oy, oz);
    E.y = interp_lds<G, DIM, 1>(Fl, rx, iy, rz, ox, hy, oz);
    E.z = interp_lds<G, DIM, 2>(Fl, rx, ry, iz, ox, oy, hz);
    B.x = interp_lds<G, DIM, 3>(Fl, rx, iy, iz, ox, hy, hz);
    B.y = interp_lds<G, DIM, 4>(Fl, ix, ry, iz, hx, oy, hz);
    B.z = interp_lds<G, DIM, 5>(Fl, ix, iy, rz, hx, hy, oz);
}

// Stage field component F (and the ones after it) of the tile into its LDS region.
template <class G, int DIM, int F, int NT>
__device__ inline void stage_fields(float* __restrict__ Fl, const StepDev& P, const int t0[3],
                                    const int ext[3], int tid)
{
    constexpr int X = G::fdim(F, 0), Y = G::fdim(F, 1), Z = G::fdim(F, 2);
    constexpr int hx = yee_half(F, 0), hy = yee_half(F, 1), hz = DIM == 3 && yee_half(F, 2);
    const float* src = F < 3 ? P.E[F] : P.B[F - 3];
    for (int e = tid; e < X * Y * Z; e += NT) {
        const int lx = e % X, ly = (e / X) % Y, lz = e / (X * Y);
        float v = 0.f;
        if (lx < ext[0] + 1 + hx && ly < ext[1] + 1 + hy && (DIM == 2 || lz < ext[2] + 1 + hz)) {
            const int64_t g = (int64_t)(t0[0] - hx + lx) + (int64_t)P.sy * (t0[1] - hy + ly) +
                              (DIM == 3 ? (int64_t)P.sz * (t0[2] - hz + lz) : 0);
            v = src[g];
        }
        Fl[G::foff(F) + e] = v;
    }
    if constexpr (F < 5) stage_fields<G, DIM, F + 1, NT>(Fl, P, t0, ext, tid);
}

// ------------------------------------------------------------------ the fused kernel
template <int DIM>
__device__ inline void tile_origin(const StepDev& P, int tile, int t0[3], int ext[3])
{
    const int tx = tile % P.tl.nt[0];
    const int r = tile / P.tl.nt[0];
    const int ty = r % P.tl.nt[1];
    const int tz = r / P.tl.nt[1];
    const int tc[3] = {tx, ty, tz};
#pragma unroll
    for (int d = 0; d < 3; d++) {
        t0[d] = tc[d] << P.tl.lt[d];
        const int e = P.n[d] - t0[d];
        ext[d] = e < (1 << P.tl.lt[d]) ? e : (1 << P.tl.lt[d]);
    }
    if (DIM == 2) {
        t0[2] = 0;
        ext[2] = 1;
    }
}

__device__ inline void latch(uint32_t* err, uint32_t bit) { atomicOr(err, bit); }

// int64 fixed-point tile sum -> FP32 current
__device__ inline float fixed_to_float(unsigned long long a, float unit)
{
    const long long v = (long long)a;
    const int hi = (int)(v >> 32);
    const unsigned lo = (unsigned)v;
    return (float)(((double)hi * 4294967296.0 + (double)lo) * (double)unit);
}

// Flush the tile current (interior + deposit halo) to the global arrays with float atomics.
template <class G, int DIM, int NT>
__device__ inline void flush_current(const unsigned long long* __restrict__ Jl, const StepDev& P,
                                     const int t0[3], const int ext[3], int tid)
{
    for (int e = tid; e < G::JTOT; e += NT) {
        const unsigned long long a = Jl[e];
        if (a == 0ull) continue;
        const int c = (e >= G::joff(1)) + (e >= G::joff(2));
        const int r = e - (c == 0 ? 0 : (c == 1 ? G::joff(1) : G::joff(2)));
        const int X = c == 0 ? G::jdim(0, 0) : (c == 1 ? G::jdim(1, 0) : G::jdim(2, 0));
        const int Y = c == 0 ? G::jdim(0, 1) : (c == 1 ? G::jdim(1, 1) : G::jdim(2, 1));
        const int lx = r % X, ly = (r / X) % Y, lz = r / (X * Y);
        if (lx < ext[0] + (c == 0 ? 2 : 3) && ly < ext[1] + (c == 1 ? 2 : 3) &&
            (DIM == 2 || lz < ext[2] + (c == 2 ? 2 : 3))) {
            const int64_t g = (int64_t)(t0[0] - 1 + lx) + (int64_t)P.sy * (t0[1] - 1 + ly) +
                              (DIM == 3 ? (int64_t)P.sz * (t0[2] - 1 + lz) : 0);
            unsafeAtomicAdd(&P.J[c][g], fixed_to_float(a, P.junit));
        }
    }
}

template <class G, int DIM>
__device__ inline LdsAcc<G> lds_acc(unsigned long long* Jl, int bx, int by, int bz)
{
    LdsAcc<G> acc;
    acc.J = Jl;
#pragma unroll
    for (int c = 0; c < 3; c++) {
        // 24-bit multiply-adds; region indices are non-negative
        unsigned b = (unsigned)bx + __umul24((unsigned)G::jdim(c, 0), (unsigned)by) +
                     (DIM == 3 ? __umul24((unsigned)(G::jdim(c, 0) * G::jdim(c, 1)), (unsigned)bz) : 0u);
        acc.base[c] = (int)b;
    }
    return acc;
}

template <int DIM, int TX, int TY, int TZ, int FRAME, int NT>
__device__ __attribute__((always_inline)) inline void gpd_body(const StepDev& P, int blk, int nblk,
                                                                int fuse)
{
    using G = Geo<DIM, TX, TY, TZ>;
    __shared__ __attribute__((aligned(16))) unsigned char lds[G::LDS_BYTES];
    float* const Fl = reinterpret_cast<float*>(lds);                                      // E, B
    unsigned long long* const Jl = reinterpret_cast<unsigned long long*>(lds + G::FBYTES);  // J

    const int tile = xcd_contiguous(blk, nblk);
    int t0[3], ext[3];
    tile_origin<DIM>(P, tile, t0, ext);
    const int tid = threadIdx.x;

    // migration counts of the next sort (per species, direction)
    __shared__ uint32_t mc[kMaxSpecies * kMigDirs];
    const int tsy = t0[1] >> P.tl.lt[1];  // y index of this tile

    stage_fields<G, DIM, 0, NT>(Fl, P, t0, ext, tid);
    if (fuse)
        for (int e = tid; e < G::JTOT; e += NT) Jl[e] = 0ull;
    if (tid < kMaxSpecies * kMigDirs) mc[tid] = 0u;
    __syncthreads();

    const int nx = P.n[0], ny = P.n[1], nz = P.n[2];
    for (int s = 0; s < P.nsp; s++) {
        const SpeciesDev& S = P.sp[s];
        bool far = false;   // a particle beyond the neighbouring tiles
        uint32_t nesc = 0;  // probabilistic escapes (one counter add per wave, at the end)
        uint32_t nsl = 0;   // shearing box: superluminal effective velocities (likewise)
        const uint32_t beg = (uint32_t)S.toff[tile], end = (uint32_t)S.toff[tile + 1];
        // the waves take 64-slot groups aligned to 32 slots (the 128-byte lines of the 4-byte
        // particle arrays), so that their stores fill whole lines; the lanes before the tile's
        // first slot idle in the first round
        for (uint32_t slot = (beg & ~31u) + tid; slot < end; slot += NT) {
            if (slot < beg) continue;
            uint32_t so = slot;
            asm("" : "+v"(so));  // keeps the 32-bit offset form (scalar base) for the stores
            const uint32_t src = (uint32_t)ld_at(S.perm, slot);
            int cx, cy, cz;
            P.cc.decode(ld_at(S.cell_in, src), cx, cy, cz);
            const float ox = ld_at(S.off_in[0], src), oy = ld_at(S.off_in[1], src);
            const float oz = DIM == 3 ? ld_at(S.off_in[2], src) : 0.f;
            f3 u = mk(ld_at(S.u_in[0], src), ld_at(S.u_in[1], src), ld_at(S.u_in[2], src));

            const int rx = cx - t0[0], ry = cy - t0[1], rz = DIM == 3 ? cz - t0[2] : 0;
            const bool in_tile = (unsigned)rx < (unsigned)ext[0] && (unsigned)ry < (unsigned)ext[1] &&
                                 (DIM == 2 || (unsigned)rz < (unsigned)ext[2]);
            f3 E, B;
            if (in_tile) {
                gather_lds<G, DIM>(Fl, rx, ry, rz, ox, oy, oz, E, B);
            } else {
                auto fa = [&](int c) -> const float* { return c < 3 ? P.E[c] : P.B[c - 3]; };
                gather<DIM>(fa, P.sy, P.sz, cx, cy, cz, ox, oy, oz, E, B);
                atomicAdd(&P.ctr[0], 1ull);
                latch(P.err, 4u);
            }

            // ---- push
            const float xr = __fadd_rn(__fsub_rn((float)cx, P.half_nx), ox);  // radial x (shearing box)
            if (FRAME == kShear)
                u = push_shear(u, E, B, S.qm_hdt, P.alpha1, P.sO * xr, P.om_dt);
            else if (FRAME == kShearExpand)
                u = push_shear_expand(u, E, B, S.qm_hdt, P.alpha1, P.sO * xr, P.om_dt, P.lam1p,
                                      P.ltil, P.tfac);
            else if (FRAME == kExpand)
                u = push_expand(u, E, B, S.qm_hdt, P.lam1p, P.ltil, P.tfac);
            else
                u = push_boris(u, E, B, S.qm_hdt);

            // ---- displacement of the deposit (comoving for the shearing box, primed for the
            // expanding box, both for the combined frame)
            const float ig = rsq1(1.f + dot(u, u));
            const float hs = P.dt * ig;
            f3 D = hs * u;
            if (frame_expanding(FRAME)) D = mk(D.x * P.linv[0], D.y * P.linv[1], D.z * P.linv[2]);
            // y increment of the position: the shearing box adds the shear move
            // y -= s Omega0 (x' + x^n)/2 dt (Sec. 2.2), x' + x^n = 2 x^n + D.x, each operation
            // rounded as written (the FP32 integer layer of the oracle repeats it bit for bit)
            float dyt = D.y, vs = 0.f;
            if (frame_sheared(FRAME)) {  // the combined frame: x and y scale together
                vs = __fmul_rn(-P.sO, __fmaf_rn(0.5f, D.x, xr));  // v_s at the midpoint x
                dyt = __fmaf_rn(P.dt, vs, D.y);
            }
            // one test catches both: a non-finite momentum makes D NaN, which fails every
            // comparison; a finite one fails it when a deposit displacement reaches half a cell
            // or the shear move takes the y increment to a whole cell (the offset
            // renormalisation needs |increment| < 1)
            if (!(fabsf(D.x) < 0.5f && fabsf(D.y) < 0.5f && (DIM == 2 || fabsf(D.z) < 0.5f) &&
                  fabsf(dyt) < 1.f))
                latch(P.err, (isfinite(u.x) && isfinite(u.y) && isfinite(u.z)) ? 1u : 2u);

            // ---- deposit xn -> xn + D
            if (fuse) {
                const int hx = ox >= 0.5f, hy = oy >= 0.5f, hz = DIM == 3 ? (oz >= 0.5f) : 0;
                const float x0 = ox - (float)hx, y0 = oy - (float)hy, z0 = oz - (float)hz;
                const Shape3 SX = shape3(x0, x0 + D.x), SY = shape3(y0, y0 + D.y);
                const Shape3 SZ = DIM == 3 ? shape3(z0, z0 + D.z) : Shape3{{0, 1, 0}, {0, 0, 0}, 0.f, 0.f};
                if (in_tile) {
                    LdsAcc<G> acc = lds_acc<G, DIM>(Jl, rx + hx, ry + hy, rz + hz);
                    esirkepov<DIM>(acc, SX, SY, SZ, S.q_dt * P.jscale, D.z);
                } else {
                    GlobalAcc acc{P.J, (int64_t)(cx + hx - 1) + (int64_t)P.sy * (cy + hy - 1) +
                                           (DIM == 3 ? (int64_t)P.sz * (cz + hz - 1) : 0),
                                  P.sy, P.sz};
                    esirkepov<DIM>(acc, SX, SY, SZ, S.q_dt, D.z);
                }
            } else {
                st_at(S.ws_cell, so, P.cc.encode(cx, cy, cz));
                st_at(S.ws_off[0], so, ox);
                st_at(S.ws_off[1], so, oy);
                if (DIM == 3) st_at(S.ws_off[2], so, oz);
                st_at(S.ws_disp[0], so, D.x);
                st_at(S.ws_disp[1], so, D.y);
                st_at(S.ws_disp[2], so, D.z);
            }

            // ---- new position: x' = x^n + D, then (shearing box) the shear move
            // y -= s Omega0 (x' + x^n)/2 dt (Sec. 2.2)
            if (frame_sheared(FRAME)) {
                // the effective velocity u'/gamma' + v_s e_y (eq. OAx) can exceed c for
                // relativistic particles (Sec. 2.1): counted, not corrected.  With
                // |u'|^2/gamma'^2 = 1 - 1/gamma'^2, |v|^2 > 1 reads vs (2 u'_y/gamma' + vs) > 1/gamma'^2.
                if (P.count_sl) nsl += (vs * fmaf(2.f * u.y, ig, vs) > ig * ig) ? 1u : 0u;
            }
            int dcx, dcy, dcz = 0;
            const float nox = renorm(__fadd_rn(ox, D.x), dcx);
            float noy = renorm(__fadd_rn(oy, dyt), dcy);
            const float noz = DIM == 3 ? renorm(__fadd_rn(oz, D.z), dcz) : 0.f;
            int ncx = cx + dcx, ncy = cy + dcy, ncz = cz + dcz;
            const bool xwrap = ncx >= nx || ncx < 0;
            if (xwrap) {
                // shearing-periodic x (Sec. 2.1): leaving through x_o re-enters at x_i with
                // y + Delta y_s(t^{n+1}); leaving through x_i re-enters at x_o with y - Delta y_s
                const bool out = ncx >= nx;
                ncx += out ? -nx : nx;
                if (frame_sheared(FRAME)) {
                    int d2;
                    noy = renorm(__fadd_rn(noy, out ? P.dys_frac : -P.dys_frac), d2);
                    // ncy in [-1, ny], dys_int in [0, ny): the sum lies in (-ny-2, 2ny+1)
                    ncy += (out ? P.dys_int : -P.dys_int) + d2;
                    if (ncy >= ny) ncy -= ny;
                    if (ncy < 0) ncy += ny;
                }
            }
            if (ncy >= ny) ncy -= ny;
            if (ncy < 0) ncy += ny;
            if (DIM == 3) {
                if (ncz >= nz) ncz -= nz;
                if (ncz < 0) ncz += nz;
            }
            int32_t ncell = P.cc.encode(ncx, ncy, ncz);

            // ---- leaky box (Sec. 4.1); in the shearing and expanding frames on request, with the
            // displacement D of the deposit: comoving (relative to the shear flow), or primed
            if (FRAME == kLeaky || (FRAME != kPlain && P.escape)) {
                const uint32_t pid = ld_at(S.id_in, src);
                if (P.leaky_mode == 0) {
                    // the z displacement is tracked only for the 3-vector test
                    float rx = ld_at(S.dr_in[0], src) + D.x, ry = ld_at(S.dr_in[1], src) + D.y;
                    float rz = 0.f;
                    float m = fmaxf(fabsf(rx), fabsf(ry));
                    if (P.use_3vec) {
                        rz = ld_at(S.dr_in[2], src) + D.z;
                        m = fmaxf(m, fabsf(rz));
                    }
                    if (m >= P.l_esc) {
                        uint32_t w[4] = {pid, P.step_lo, 1u, P.box_id};
                        philox4x32_10(w, P.key0, P.key1);
                        // inverse CDF of |u| (bulk bins linear in p, top bin linear in -log2(1-p))
                        const uint32_t bin = w[0] >> 20, rr = w[0] & 0xFFFFFu;
                        float um;
                        if (bin < (uint32_t)(kMjBins - 1)) {
                            const float fr = (float)rr * (1.f / 1048576.f);
                            um = P.mj[bin] + fr * (P.mj[bin + 1] - P.mj[bin]);
                        } else {
                            const float sv = 20.f - log2f((float)(0x100000u - rr));
                            const float xk = sv * ((float)kMjTail / 20.f);
                            int k = (int)xk;
                            k = k > kMjTail - 1 ? kMjTail - 1 : k;
                            const float fr = xk - (float)k;
                            const float* T = P.mj + kMjBins - 1;
                            um = T[k] + fr * (T[k + 1] - T[k]);
                        }
                        const float mu = 2.f * ((float)(w[1] >> 8) * (1.f / 16777216.f)) - 1.f;
                        const float phi = 6.283185307179586f * ((float)(w[2] >> 8) * (1.f / 16777216.f));
                        float sp, cp;
                        sincosf(phi, &sp, &cp);
                        const float st = sqrtf(fmaxf(0.f, 1.f - mu * mu));
                        u = mk(um * st * cp, um * st * sp, um * mu);
                        rx = ry = rz = 0.f;
                    }
                    st_at(S.dr_out[0], so, rx);
                    st_at(S.dr_out[1], so, ry);
                    if (P.use_3vec) st_at(S.dr_out[2], so, rz);
                } else {
                    const double g2m1 = ((double)u.x * (double)u.x + (double)u.y * (double)u.y) +
                                        (double)u.z * (double)u.z;
                    if (g2m1 > P.g2thr) {
                        uint32_t w[4] = {pid, P.step_lo, 0u, P.box_id};
                        philox4x32_10(w, P.key0, P.key1);
                        if (w[0] < P.esc_thr) {
                            ncell = -1;
                            nesc++;
                        }
                    }
                }
            }

            if (P.count_mig) {
                // direction of the new tile from this one (the migration sort applies only to
                // whole tiles): the cell step r + dc in [-1, edge] shifted right by log2(edge)
                // is -1, 0 or +1, periodic wraps included; one tile on an axis means 0.  A
                // shearing-box x-face crossing moves in y by the push's Delta y_s: its y step is
                // taken against the tile shift of that face.
                const int dx = P.mg.nt[0] == 1 ? 0 : (rx + dcx) >> P.tl.lt[0];
                int dy = P.mg.nt[1] == 1 ? 0 : (ry + dcy) >> P.tl.lt[1];
                const int dz = (DIM == 2 || P.mg.nt[2] == 1) ? 0 : (rz + dcz) >> P.tl.lt[2];
                if (frame_sheared(FRAME) && xwrap && P.mg.nt[1] > 1) {
                    int r = (ncy >> P.tl.lt[1]) - tsy - (dx > 0 ? P.mg.cy_out : P.mg.cy_in);
                    const int n1 = P.mg.nt[1];  // r lies in (-2 n1, 2 n1)
                    if (r < 0) r += n1;
                    if (r < 0) r += n1;
                    if (r >= n1) r -= n1;
                    dy = r == 0 ? 0 : (r == 1 ? 1 : (r == n1 - 1 ? -1 : 2));
                }
                int d = dy == 2 ? -1 : (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
                if (ncell < 0) d = kMigDead;
                // the particles that stay in the tile (the common direction, 13) are not counted
                // here: they are the tile's particles less all the others (below)
                if (d != 13) {
                    if (d >= 0)
                        atomicAdd(&mc[s * kMigDirs + d], 1u);
                    else
                        far = true;
                }
            }
            st_at(S.cell_out, so, ncell);
            st_at(S.off_out[0], so, nox);
            st_at(S.off_out[1], so, noy);
            if (DIM == 3) st_at(S.off_out[2], so, noz);
            st_at(S.u_out[0], so, u.x);
            st_at(S.u_out[1], so, u.y);
            st_at(S.u_out[2], so, u.z);
            if (P.track_ids) st_at(S.id_out, so, ld_at(S.id_in, src));
        }
        if (FRAME == kLeaky || (FRAME != kPlain && P.escape)) {
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) nesc += __shfl_xor(nesc, o, 64);
            if ((tid & 63) == 0 && nesc) atomicAdd(&P.ctr[1], (unsigned long long)nesc);
        }
        if (frame_sheared(FRAME) && P.count_sl) {
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) nsl += __shfl_xor(nsl, o, 64);
            if ((tid & 63) == 0 && nsl) atomicAdd(&P.ctr[3], (unsigned long long)nsl);
        }
        if (P.count_mig) {
            if (far) {
                *P.mfb[s] = 1;
                if (P.mig_latch) latch(P.err, kErrSort);
            }
        }
    }

    if (!fuse && !P.count_mig) return;
    __syncthreads();
    if (P.count_mig && tid < P.nsp * kMigDirs) {
        const int s = tid / kMigDirs, d = tid - s * kMigDirs;
        uint32_t v = mc[tid];
        if (d == 13) {  // the stayers: every particle of the tile goes to exactly one direction
            v = (uint32_t)(P.sp[s].toff[tile + 1] - P.sp[s].toff[tile]);
            for (int e = 0; e < kMigDirs; e++)
                if (e != 13) v -= mc[s * kMigDirs + e];
        }
        P.mcnt[s][(size_t)tile * kMigDirs + d] = v;
    }
    if (fuse) flush_current<G, DIM, NT>(Jl, P, t0, ext, tid);
}

// 3D tiles: compact regions (48.4 KB of LDS for 8^3) let three workgroups share a CU, so the
// register budget is set for 6 waves per SIMD.  2D tiles of 16x16 and 8x8 (16 KB and less) fit
// eight waves per SIMD in 64 VGPRs (a few spilled: 2-4 % faster for the leaky box than at the
// 81-93 VGPRs of no budget); the larger 2D tiles are bound by their LDS first.
template <int DIM, int TX, int TY, int TZ, int FRAME, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(DIM == 3 ? 6 : 8)))
void gpd_kernel(StepDev P, int fuse)
{
    gpd_body<DIM, TX, TY, TZ, FRAME, NT>(P, (int)blockIdx.x, (int)gridDim.x, fuse);
}

// Many boxes in one launch: the blocks of unit u (one box's tiles) take its descriptor.
template <int DIM, int TX, int TY, int TZ, int FRAME, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(DIM == 3 ? 6 : 8)))
void gpd_batch(const StepDev* __restrict__ t, UnitMap m)
{
    const int u = unit_of(m, (int)blockIdx.x);
    gpd_body<DIM, TX, TY, TZ, FRAME, NT>(t[u], (int)blockIdx.x - (int)m.prefix[u],
                                         (int)(m.prefix[u + 1] - m.prefix[u]), 1);
}

// Unfused deposit: the same Esirkepov tile accumulation from the positions and deposit
// displacements saved by an unfused push (in sorted slot order).
template <int DIM, int TX, int TY, int TZ, int NT>
__global__ __launch_bounds__(NT) void deposit_kernel(StepDev P)
{
    using G = Geo<DIM, TX, TY, TZ>;
    __shared__ unsigned long long Jl[G::JTOT];
    const int tile = xcd_contiguous(blockIdx.x, gridDim.x);
    int t0[3], ext[3];
    tile_origin<DIM>(P, tile, t0, ext);
    const int tid = threadIdx.x;
    for (int e = tid; e < G::JTOT; e += NT) Jl[e] = 0ull;
    __syncthreads();
    for (int s = 0; s < P.nsp; s++) {
        const SpeciesDev& S = P.sp[s];
        const uint32_t beg = (uint32_t)S.toff[tile], end = (uint32_t)S.toff[tile + 1];
        for (uint32_t slot = beg + tid; slot < end; slot += NT) {
            int cx, cy, cz;
            P.cc.decode(ld_at(S.ws_cell, slot), cx, cy, cz);
            const float ox = ld_at(S.ws_off[0], slot), oy = ld_at(S.ws_off[1], slot);
            const float oz = DIM == 3 ? ld_at(S.ws_off[2], slot) : 0.f;
            const f3 D = mk(ld_at(S.ws_disp[0], slot), ld_at(S.ws_disp[1], slot),
                            ld_at(S.ws_disp[2], slot));
            const int rx = cx - t0[0], ry = cy - t0[1], rz = DIM == 3 ? cz - t0[2] : 0;
            const bool in_tile = (unsigned)rx < (unsigned)ext[0] && (unsigned)ry < (unsigned)ext[1] &&
                                 (DIM == 2 || (unsigned)rz < (unsigned)ext[2]);
            const int hx = ox >= 0.5f, hy = oy >= 0.5f, hz = DIM == 3 ? (oz >= 0.5f) : 0;
            const float x0 = ox - (float)hx, y0 = oy - (float)hy, z0 = oz - (float)hz;
            const Shape3 SX = shape3(x0, x0 + D.x), SY = shape3(y0, y0 + D.y);
            const Shape3 SZ = DIM == 3 ? shape3(z0, z0 + D.z) : Shape3{{0, 1, 0}, {0, 0, 0}, 0.f, 0.f};
            if (in_tile) {
                LdsAcc<G> acc = lds_acc<G, DIM>(Jl, rx + hx, ry + hy, rz + hz);
                esirkepov<DIM>(acc, SX, SY, SZ, S.q_dt * P.jscale, D.z);
            } else {
                GlobalAcc acc{P.J, (int64_t)(cx + hx - 1) + (int64_t)P.sy * (cy + hy - 1) +
                                       (DIM == 3 ? (int64_t)P.sz * (cz + hz - 1) : 0),
                              P.sy, P.sz};
                esirkepov<DIM>(acc, SX, SY, SZ, S.q_dt, D.z);
            }
        }
    }
    __syncthreads();
    flush_current<G, DIM, NT>(Jl, P, t0, ext, tid);
}

// ------------------------------------------------------------------ launchers
// threads per workgroup: 3D tiles hold a 56 KB LDS footprint (2 workgroups per CU), so they
// use 8 waves per workgroup to keep 16 waves per CU
template <int DIM>
constexpr int threads_for() { return DIM == 3 ? 512 : 256; }

template <int DIM, int TX, int TY, int TZ>
static hipError_t launch_shape(const StepDev& P, int fuse, hipStream_t st)
{
    constexpr int NT = threads_for<DIM>();
    const dim3 grid(P.tl.n_tiles), block(NT);
    switch (P.frame) {
    case kShear:
        gpd_kernel<DIM, TX, TY, TZ, kShear, NT><<<grid, block, 0, st>>>(P, fuse);
        break;
    case kExpand:
        gpd_kernel<DIM, TX, TY, TZ, kExpand, NT><<<grid, block, 0, st>>>(P, fuse);
        break;
    case kLeaky:
        gpd_kernel<DIM, TX, TY, TZ, kLeaky, NT><<<grid, block, 0, st>>>(P, fuse);
        break;
    case kShearExpand:
        gpd_kernel<DIM, TX, TY, TZ, kShearExpand, NT><<<grid, block, 0, st>>>(P, fuse);
        break;
    default:
        gpd_kernel<DIM, TX, TY, TZ, kPlain, NT><<<grid, block, 0, st>>>(P, fuse);
        break;
    }
    return hipGetLastError();
}

template <int DIM, int TX, int TY, int TZ>
static hipError_t launch_dep_shape(const StepDev& P, hipStream_t st)
{
    constexpr int NT = threads_for<DIM>();
    deposit_kernel<DIM, TX, TY, TZ, NT><<<dim3(P.tl.n_tiles), dim3(NT), 0, st>>>(P);
    return hipGetLastError();
}

// Tile shapes (edges in cells) with an instantiated fused kernel, and the subset the batched
// launch supports.  Returns the number of shapes written (at most max).
int tile_candidates(int dim, bool batched, int (*out)[3], int max)
{
    static const int k3[][3] = {{8, 8, 8}, {4, 4, 4}};
    static const int k2[][3] = {{16, 16, 1}, {8, 8, 1}, {32, 16, 1}, {32, 32, 1}};
    const int (*list)[3] = dim == 3 ? k3 : k2;
    const int n = dim == 3 ? (batched ? 1 : 2) : (batched ? 2 : 4);
    int w = 0;
    for (int i = 0; i < n && w < max; i++, w++)
        for (int k = 0; k < 3; k++) out[w][k] = list[i][k];
    return w;
}

static bool in_candidates(int dim, bool batched, const int t[3])
{
    int c[8][3];
    const int n = tile_candidates(dim, batched, c, 8);
    for (int i = 0; i < n; i++)
        if (c[i][0] == t[0] && c[i][1] == t[1] && c[i][2] == t[2]) return true;
    return false;
}

bool tile_shape_supported(int dim, const int t[3]) { return in_candidates(dim, false, t); }

template <int DIM, int TX, int TY, int TZ>
static hipError_t launch_batch_shape(const StepDev* table, UnitMap m, int blocks, int frame,
                                     hipStream_t st)
{
    constexpr int NT = threads_for<DIM>();
    switch (frame) {
    case kShear: gpd_batch<DIM, TX, TY, TZ, kShear, NT><<<blocks, NT, 0, st>>>(table, m); break;
    case kExpand: gpd_batch<DIM, TX, TY, TZ, kExpand, NT><<<blocks, NT, 0, st>>>(table, m); break;
    case kShearExpand: gpd_batch<DIM, TX, TY, TZ, kShearExpand, NT><<<blocks, NT, 0, st>>>(table, m); break;
    case kLeaky: gpd_batch<DIM, TX, TY, TZ, kLeaky, NT><<<blocks, NT, 0, st>>>(table, m); break;
    default: gpd_batch<DIM, TX, TY, TZ, kPlain, NT><<<blocks, NT, 0, st>>>(table, m); break;
    }
    return hipGetLastError();
}

bool batch_tile_supported(int dim, const int t[3]) { return in_candidates(dim, true, t); }

hipError_t launch_gather_push_batch(const StepDev* table, UnitMap m, int blocks, int dim,
                                    const int t[3], int frame, hipStream_t st)
{
    if (blocks <= 0) return hipSuccess;
    if (dim == 3) return launch_batch_shape<3, 8, 8, 8>(table, m, blocks, frame, st);
    if (t[0] == 16) return launch_batch_shape<2, 16, 16, 1>(table, m, blocks, frame, st);
    return launch_batch_shape<2, 8, 8, 1>(table, m, blocks, frame, st);
}

hipError_t launch_gather_push(const StepDev& P, const int t[3], int fuse, hipStream_t st)
{
    if (P.dim == 3) {
        if (t[0] == 8) return launch_shape<3, 8, 8, 8>(P, fuse, st);
        return launch_shape<3, 4, 4, 4>(P, fuse, st);
    }
    if (t[0] == 16) return launch_shape<2, 16, 16, 1>(P, fuse, st);
    if (t[0] == 8) return launch_shape<2, 8, 8, 1>(P, fuse, st);
    if (t[1] == 16) return launch_shape<2, 32, 16, 1>(P, fuse, st);
    return launch_shape<2, 32, 32, 1>(P, fuse, st);
}

hipError_t launch_deposit(const StepDev& P, const int t[3], hipStream_t st)
{
    if (P.dim == 3) {
        if (t[0] == 8) return launch_dep_shape<3, 8, 8, 8>(P, st);
        return launch_dep_shape<3, 4, 4, 4>(P, st);
    }
    if (t[0] == 16) return launch_dep_shape<2, 16, 16, 1>(P, st);
    if (t[0] == 8) return launch_dep_shape<2, 8, 8, 1>(P, st);
    if (t[1] == 16) return launch_dep_shape<2, 32, 16, 1>(P, st);
    return launch_dep_shape<2, 32, 32, 1>(P, st);
}

}  // namespace pic
