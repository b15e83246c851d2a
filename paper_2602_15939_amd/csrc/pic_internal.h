// pic_internal.h — device-side layout shared by the HIP kernels and the host driver of
// the particle hot path (gfx950).  Not part of the public C ABI (include/pic.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pic {

constexpr int kGuard = 2;      // guard cells on each side of every grid axis (z: 0 in 2D)
constexpr int kMaxSpecies = 2;
constexpr int kBlock = 256;    // threads per workgroup of the particle kernels (4 wave64)
constexpr int kMjBins = 4096;  // reinjection sampler: bulk inverse-CDF bins
constexpr int kMjTail = 64;    // reinjection sampler: tail bins in -log2(1-p)

enum Frame { kPlain = 0, kShear = 1, kExpand = 2, kLeaky = 3, kShearExpand = 4 };
// frames with the shearing-box geometry, and with the expanding-box scale factors
constexpr bool frame_sheared(int f) { return f == kShear || f == kShearExpand; }
constexpr bool frame_expanding(int f) { return f == kExpand || f == kShearExpand; }

// Particle cells are packed as i | j << b0 | k << (b0+b1) with b_d = ceil(log2 n_d),
// so decoding is shifts and masks.  A dead particle has cell -1.
struct CellCode {
    int b0, b1;
    unsigned m0, m1;
    __host__ __device__ inline void decode(int32_t c, int& i, int& j, int& k) const
    {
        unsigned u = (unsigned)c;
        i = (int)(u & m0);
        j = (int)((u >> b0) & m1);
        k = (int)(u >> (b0 + b1));
    }
    __host__ __device__ inline int32_t encode(int i, int j, int k) const
    {
        return (int32_t)((unsigned)i | ((unsigned)j << b0) | ((unsigned)k << (b0 + b1)));
    }
};

// Geometry of the tile decomposition (power-of-two tile edges).
struct Tiles {
    int lt[3];    // log2 of the tile edge per axis
    int nt[3];    // tiles per axis
    int n_tiles;
    __host__ __device__ inline int key(int i, int j, int k) const
    {
        return (i >> lt[0]) + nt[0] * ((j >> lt[1]) + nt[1] * (k >> lt[2]));
    }
};

// Directions of the migration sort: (dx, dy, dz) in {-1,0,1}^3 between the tile a particle
// was sorted into and the tile of its new cell, index (dx+1) + 3 (dy+1) + 9 (dz+1); the last
// direction is the dead bin.  Crossing the x faces of the shearing box shifts y by the tile
// offset cy_out (leaving through the outer face) or cy_in (inner face) before dy is taken.
constexpr int kMigDirs = 28;
constexpr uint32_t kErrSort = 16u;  // a batched sort met a particle beyond the neighbour tiles
constexpr uint32_t kErrNoConverge = 32u;  // shearing-box sweeps missed their tolerance
constexpr int kMigDead = 27;
struct MigGeo {
    int nt[3], lt[3];
    int n_tiles;
    int cy_out, cy_in;
};

// d in (-2n, 2n) reduced on a ring of n tiles to -1, 0, +1, or 2 if it is farther (conditional
// adds: no integer division)
__device__ inline int ring_step(int d, int n)
{
    if (n == 1) return 0;
    int r = d;
    if (r < 0) r += n;
    if (r < 0) r += n;
    if (r >= n) r -= n;
    if (r == 0) return 0;
    if (r == 1) return 1;
    if (r == n - 1) return -1;
    return 2;
}

__device__ inline void tile_coords(const MigGeo& g, int t, int& x, int& y, int& z)
{
    x = t % g.nt[0];
    const int r = t / g.nt[0];
    y = r % g.nt[1];
    z = r / g.nt[1];
}

// direction of a particle of source tile (sx, sy, sz) with new cell c, or -1 if its new tile is
// not a neighbour
__device__ inline int mig_dir(const MigGeo& g, const CellCode& cc, int sx, int sy, int sz,
                              int32_t c)
{
    if (c < 0) return kMigDead;
    int x, y, z;
    cc.decode(c, x, y, z);
    const int tx = x >> g.lt[0], ty = y >> g.lt[1], tz = z >> g.lt[2];
    int dx = tx - sx, wx = 0;
    if (g.nt[0] == 1) {
        dx = 0;
    } else if (dx == g.nt[0] - 1 && dx > 1) {  // through the inner x face
        dx = -1;
        wx = -1;
    } else if (dx == 1 - g.nt[0] && dx < -1) {  // through the outer x face
        dx = 1;
        wx = 1;
    } else if (dx < -1 || dx > 1) {
        return -1;
    }
    // tiles and the shifts lie in [0, nt): the differences below lie in (-2 nt, nt)
    const int shift = wx > 0 ? g.cy_out : (wx < 0 ? g.cy_in : 0);
    const int dy = ring_step(ty - sy - shift, g.nt[1]);
    const int dz = ring_step(tz - sz, g.nt[2]);
    if (dy == 2 || dz == 2) return -1;
    return (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
}

// One species as seen by a push launch: input arrays (read through perm), output arrays
// (written in sorted slot order) and the unfused-deposit workspace.
struct SpeciesDev {
    const int32_t* cell_in;
    const float* off_in[3];
    const float* u_in[3];
    const uint32_t* id_in;
    const float* dr_in[3];
    int32_t* cell_out;
    float* off_out[3];
    float* u_out[3];
    uint32_t* id_out;
    float* dr_out[3];
    const int32_t* perm;  // sorted slot -> input index
    const int32_t* toff;  // tile offsets, n_tiles + 1
    int32_t* ws_cell;     // unfused deposit: old cell, old offsets, deposit displacement
    float* ws_off[3];
    float* ws_disp[3];
    float qm_hdt;         // (q/m) dt/2
    float q_dt;           // macro charge / dt
};

// Everything one push or deposit launch of one box needs, passed by value.
struct StepDev {
    int dim, frame;
    int n[3];
    CellCode cc;
    Tiles tl;
    int sy, sz;           // element strides of the guarded grid arrays (x stride 1)
    float* E[3];          // pointers to interior (0,0,0) of the guarded arrays
    float* B[3];
    float* J[3];
    float dt;
    // shearing box
    float sO;             // s Omega0
    float om_dt;          // Omega0 dt
    float alpha1;         // s Omega0 dt/2
    float half_nx;        // n[0]/2
    int dys_int;          // Delta y_s(t^{n+1}) = dys_int + dys_frac, dys_frac in [0,1)
    float dys_frac;
    // expanding box (Lambda at t^n, L^-1 at t^{n+1/2})
    float lam1p[3];       // 1 + Lambda_ii
    float ltil[3];        // (1 + Lambda_ii)/(1 - Lambda_ii)
    float tfac[3];        // 1/(1 - Lambda_ii)
    float linv[3];        // 1/l_i(t^{n+1/2})
    // leaky box
    int leaky_mode, use_3vec;
    int escape;  // the leaky box's escape rule applies (always in the leaky frame; on request
                 // in the shearing and expanding frames)
    float l_esc;
    uint32_t esc_thr;     // floor((dt/t_esc) 2^32)
    double g2thr;         // gamma_thr^2 - 1
    uint32_t key0, key1, step_lo, box_id;
    const float* mj;      // kMjBins + kMjTail values
    // fixed-point tile current: contribution * jscale -> integer units, units * junit -> J
    float jscale, junit;
    // migration counts of the next sort, taken by the push: per species and source tile
    // (= this launch's tile), the particles per direction (mcnt[tile * kMigDirs + d]); a
    // particle beyond the neighbouring tiles sets mfb (the radix fallback runs then)
    int count_mig;
    int mig_latch;  // batched steps (no radix fallback behind the sort): latch kErrSort too
    MigGeo mg;
    uint32_t* mcnt[kMaxSpecies];
    int32_t* mfb[kMaxSpecies];
    // bookkeeping
    uint32_t* err;
    unsigned long long* ctr;  // [0] slow-path particles, [1] escapes
    int nsp;
    int track_ids;
    int count_sl;  // shearing box: count superluminal effective velocities (PIC_BOX_COUNT_SUPERLUMINAL)
    SpeciesDev sp[kMaxSpecies];
};

// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11): ten rounds of the two 32x32->64
// multiplications with the published multipliers, key bumped by the published Weyl
// constants between rounds.
__device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; r++) {
        const uint32_t a0 = c[0], a2 = c[2];
        const uint32_t hi0 = __umulhi(0xD2511F53u, a0), lo0 = 0xD2511F53u * a0;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, a2), lo1 = 0xCD9E8D57u * a2;
        c[0] = hi1 ^ c[1] ^ k0;
        c[1] = lo1;
        c[2] = hi0 ^ c[3] ^ k1;
        c[3] = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Maps block b of a grid of nblk blocks to a work index so that each of the 8 XCDs (which
// receive blocks round-robin) processes one contiguous range of tiles and shares its L2
// for the overlapping tile halos.
__device__ inline int xcd_contiguous(int b, int nblk)
{
    const int x = b & 7, local = b >> 3;
    const int full = nblk >> 3, rem = nblk & 7;
    return x * full + (x < rem ? x : rem) + local;
}

// ---- batched launches
// One launch runs the blocks of many independent work units (boxes, or parts of boxes):
// prefix[u] is the first block of unit u, prefix[nu] the total.  A kernel body takes its unit's
// arguments, its block index inside the unit, the unit's block count and blockIdx.y.
struct UnitMap {
    const uint32_t* prefix;
    int nu;
};
__device__ inline int unit_of(const UnitMap& m, int b)  // the unit owning block b
{
    int lo = 0, hi = m.nu;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if ((int)m.prefix[mid] <= b)
            lo = mid;
        else
            hi = mid;
    }
    return __builtin_amdgcn_readfirstlane(lo);  // uniform: descriptor loads stay scalar
}
// name##_kernel(Args): one unit, arguments by value; name##_batch(table, map): many units.
#define PIC_BATCHED_KERNEL(name, Args, NT)                                                       \
    __global__ __launch_bounds__(NT) void name##_kernel(Args a)                                  \
    {                                                                                            \
        name##_body(a, (int)blockIdx.x, (int)gridDim.x, (int)blockIdx.y);                        \
    }                                                                                            \
    __global__ __launch_bounds__(NT) void name##_batch(const Args* __restrict__ t, UnitMap m)   \
    {                                                                                            \
        const int u = unit_of(m, (int)blockIdx.x);                                               \
        name##_body(t[u], (int)blockIdx.x - (int)m.prefix[u], (int)(m.prefix[u + 1] - m.prefix[u]), \
                    (int)blockIdx.y);                                                            \
    }

// Geometry of a guarded grid array.
// Division of 32-bit unsigned integers by an invariant divisor d >= 1 (Granlund and Montgomery,
// "Division by invariant integers using multiplication", PLDI 1994, Fig. 4.1): with
// l = ceil(log2 d) and m = floor(2^32 (2^l - d) / d) + 1, q = (t1 + ((t - t1) >> 1)) >> (l - 1),
// t1 = mulhi(m, t), for every t < 2^32 and d >= 2; d = 1 is q = t.
struct FastDiv {
    uint32_t m;
    int l;  // 0 for d = 1
    static FastDiv make(uint32_t d)
    {
        FastDiv f{0u, 0};
        while ((1ull << f.l) < d) f.l++;
        if (f.l > 0)
            f.m = (uint32_t)((((1ull << 32) * ((1ull << f.l) - d)) / d) + 1ull);
        return f;
    }
    __device__ inline uint32_t div(uint32_t t) const
    {
        if (l == 0) return t;
        const uint32_t t1 = __umulhi(m, t);
        return (t1 + ((t - t1) >> 1)) >> (l - 1);
    }
};

struct GridDev {
    int dim;
    int n[3];
    int g[3];    // guard width per axis
    int sy, sz;  // element strides (x stride 1)
    FastDiv div0, div1;  // division by n[0] and by n[1] (linear interior index -> x, y, z)
    FastDiv divyg;       // division by the guarded row count n[1] + 2 g[1]
};

// One Yee update: X_i <- fout_i (fin_i X_i +/- dt curl(g Y)_i [- 4 pi dt J_i]).
struct MaxwellDev {
    GridDev G;
    float* E[3];
    float* B[3];
    const float* J[3];
    float dt;
    float fin[3], fout[3], gf[3];
};

// Arguments of the grid kernels (one unit each; batched launches take tables of them).
struct Comp6 {
    float* p[6];
};
struct Comp3 {
    float* p[3];
};
struct FillArgs {  // guard fill of one slab kind (0: x, 1: y, 2: z) of ncomp = gridDim.y arrays
    GridDev G;
    Comp6 A;
    int slab, shear, dys_int;
    float dys_w;
};
struct FoldPArgs {  // periodic current fold along axis 1 (y) or 2 (z)
    GridDev G;
    Comp3 J;
    int axis;
};
struct ShearFoldArgs {  // J' transport along y and shearing-periodic x fold, in -> out
    GridDev G;
    Comp3 in, out;
    float sO_hdt, half_nx;
    int dys_int;
    float dys_w;
};
struct FoldXArgs {  // x fold (periodic or shearing-periodic)
    GridDev G;
    Comp3 in, out;
    int all, shear, dys_int;
    float dys_w;
};
struct ZeroArgs {  // n 32-bit words set to zero
    uint32_t* p;
    int64_t n;
};

// One fixed-point sweep of the shearing-box implicit midpoint rule: Fo = C + dt/2 L(Fk); the
// first sweep of a step (Fk = F^n) also writes C = F^n + dt/2 L(F^n) - 4 pi dt J'.
struct KsbDev {
    GridDev G;
    const float* Fk[6];  // iterate, Bx By Bz Ex Ey Ez (guard cells filled)
    float* C[6];         // constant part of the step (written by the first sweep)
    float* Fo[6];        // next iterate (interior)
    const float* J[3];
    float dt, sO, half_nx;
    // shift of the iterate's shearing-periodic x images, Delta y_s = ydys_int + ydys_w with
    // ydys_w in [0,1) (the 3D sweep reads its x halo there instead of from guard cells)
    int ydys_int;
    float ydys_w;
    // tolerance mode (conv != nullptr): sweep k adds max|F^{k+1} - F^k| and max|F^{k+1}| (FP32
    // bit patterns, non-negative, so unsigned order is float order; NaN counts as +inf) into
    // conv[2k], conv[2k+1], which start at zero; it returns at once when the sweep before it
    // met the tolerance, leaving its pair at zero, which reads as met for the next one
    uint32_t* conv;
    float tol;
    int k;
    // two sweeps per pass (3D grids of the staged sweep, fixed sweep count): the shift of the
    // intermediate iterate's x images, Delta y_s at t^{n+1} = y1_int + y1_w
    int y1_int;
    float y1_w;
    // combined shearing and expanding frame (one-thread-per-cell sweeps only): the iterates are
    // the expanding-frame fields, the curls act on dfac[c] F_c and kz multiplies the z
    // transport of E'_y in dE'_z/dt
    int expand;
    float dfac[3];
    float kz;
};
constexpr int kKsbMaxSweeps = 64;
// words of a box's convergence record: kKsbMaxSweeps pairs, then the sweep count of the last
// step
constexpr int kKsbConvWords = 2 * kKsbMaxSweeps + 2;

// End of a tolerance-mode step: k* = the first sweep that met the tolerance (the last sweep K-1
// if none did, which latches kErrNoConverge).  The iterate of sweep k* sits in the field set
// that sweep K-1 would have written when K-1-k* is even, in the other set otherwise: then
// the interior of src (that other set) is copied to dst.
struct KsbFin {
    GridDev G;
    const uint32_t* conv;
    int32_t* sweeps;
    uint32_t* err;
    float tol;
    int K;
    const float* src[6];
    float* dst[6];
};

// Sort workspace of one species.
struct SortBufs {
    uint32_t* keys[2];
    uint32_t* vals[2];
    uint32_t* hist;
    uint32_t* scratch;
    // migration sort (kMigDirs counters per source tile, per-destination scans)
    uint32_t* mcnt;    // n_tiles * kMigDirs: particles of source tile s moving in direction d
    uint32_t* mpre;    // n_tiles * kMigDirs: offset of (s, d) inside its destination tile
    uint32_t* tot;     // n_tiles + 1: particles arriving in each tile (last entry 0)
    uint32_t* start;   // n_tiles + 1: exclusive scan of tot
    uint32_t* dcnt;    // n_tiles + 1: particles of each source tile that died (last entry 0)
    uint32_t* dpre;    // n_tiles + 1: exclusive scan of dcnt
    uint32_t* mscratch;
    int32_t* fallback; // set when a particle left the neighbourhood the migration sort covers
};

// A launch gated on a device flag runs only when *flag == want (flag == nullptr: always), so
// that a fallback path can be queued behind a test without a host round trip.
struct Gate {
    const int32_t* flag;
    int want;
    __device__ inline bool off() const { return flag && *flag != want; }
};


struct MigCountArgs {
    const int32_t* cell;
    const int32_t* toff_prev;
    CellCode cc;
    MigGeo g;
    uint32_t* mcnt;
    int32_t* fallback;
    uint32_t* err;  // batched sorts (no radix fallback behind them) latch kErrSort here
};
struct MigOffArgs {
    const uint32_t* mcnt;
    MigGeo g;
    uint32_t *mpre, *tot, *dcnt;
    Gate gate;
};
struct MigScatterArgs {
    const int32_t* cell;
    const int32_t* toff_prev;
    int n_upper;
    CellCode cc;
    MigGeo g;
    const uint32_t *mpre, *start, *dpre;
    uint32_t* perm;
    int32_t* toff;
    int32_t* n_live;
    Gate gate;
};
struct ScanArgs {  // exclusive scan of n words by one workgroup
    const uint32_t* in;
    uint32_t* out;
    int n;
    Gate gate;
};

// ---- launchers (gpd.hip, sort.hip, grid.hip, xfer.hip)
bool tile_shape_supported(int dim, const int t[3]);
// supported tile shapes (batched: those of the batched launch); the default shape comes first
int tile_candidates(int dim, bool batched, int (*out)[3], int max);
hipError_t launch_gather_push(const StepDev& P, const int t[3], int fuse, hipStream_t st);
hipError_t launch_deposit(const StepDev& P, const int t[3], hipStream_t st);
// fused push of many boxes of one dimension, tile shape and frame (table: one StepDev per box,
// m.prefix: first block of each box = its first tile)
bool batch_tile_supported(int dim, const int t[3]);
hipError_t launch_gather_push_batch(const StepDev* table, UnitMap m, int blocks, int dim,
                                    const int t[3], int frame, hipStream_t st);

size_t scan_scratch_words(int64_t n);
size_t sort_hist_words(int64_t n);
hipError_t tile_sort(const int32_t* cell, const int32_t* n_live_in, int n_upper, CellCode cc,
                     Tiles tl, SortBufs& sb, int32_t* toff, int32_t* n_live_out, int& which,
                     hipStream_t st);

// Migration sort: stable counting sort by tile of arrays still grouped by the tiles of the
// previous sort (toff_prev), every particle within one tile of its old one.  Falls back to
// tile_sort on the device when a particle is outside that neighbourhood.  Writes the
// permutation to sb.vals[which] and the offsets to toff.
size_t migrate_scratch_words(int n_tiles);
// counts_ready: the push already wrote sb.mcnt and the fallback flag (the count pass is skipped)
hipError_t migrate_sort(const int32_t* cell, const int32_t* toff_prev, int n_upper, CellCode cc,
                        Tiles tl, const MigGeo& mg, SortBufs& sb, int32_t* toff,
                        int32_t* n_live_out, int& which, unsigned long long* n_fallback,
                        bool counts_ready, hipStream_t st);

// batched launches of the grid and sort kernels (tables of per-unit arguments on the device)
// per-component factors of a field set (the combined frame's conversion to and from the
// expanding-frame fields): F_c *= f[c % 3] on the interior
struct ScaleArgs {
    GridDev G;
    float* F[6];
    float f[3];
};
enum GridBatchKind {
    kBatchZero, kBatchFill, kBatchFoldP, kBatchShearFold, kBatchFoldX, kBatchYeeB, kBatchYeeE,
    kBatchKsbFirst, kBatchKsbNext, kBatchKsbFinal, kBatchScale
};
hipError_t grid_batch(GridBatchKind k, const void* table, UnitMap m, int blocks, int ydim,
                      hipStream_t st);
unsigned grid_blocks(int64_t items);  // workgroups of kBlock threads for one item per thread
enum SortBatchKind { kBatchMigCount, kBatchMigOffsets, kBatchScan, kBatchMigScatter };
hipError_t sort_batch(SortBatchKind k, const void* table, UnitMap m, int blocks, hipStream_t st);
int sort_result_buffer(const Tiles& tl);  // sort buffer holding the sorted pairs

hipError_t fill_guards(const GridDev& G, float* const* comps, int ncomp, int shear, double dys,
                       hipStream_t st);
// Fold the current guards (y, z periodic in place).  Shearing box: the J' transport and the
// shearing-periodic x fold in one pass from J into `out` (the caller then swaps the two arrays);
// otherwise the periodic x fold in place.
hipError_t fold_current(const GridDev& G, float* const* J, float* const* out, int shear,
                        double sO, double dt, double dys_half, hipStream_t st);
hipError_t yee_b(const MaxwellDev& M, hipStream_t st);
hipError_t yee_e(const MaxwellDev& M, hipStream_t st);
// one sweep; 3D grids whose x size is a multiple of the staged kernel's column tile (128) take
// the staged kernel, which reads its whole halo at the (shearing-)periodic images itself;
// otherwise one thread per cell reads the guard cells, which must be filled between sweeps
bool ksb_staged(const GridDev& G);
// the two-sweep pass applies: a staged grid whose arrays span less than 4 GiB (32-bit offsets)
bool ksb_pass_fits(const GridDev& G);
hipError_t ksb_sweep(const KsbDev& K, bool first, hipStream_t st);
// the one-thread-per-cell sweep on any grid (reads the iterate's guard cells)
hipError_t ksb_sweep_unstaged(const KsbDev& K, bool first, hipStream_t st);
// two sweeps F^k -> F^{k+2} in one pass over memory (staged 3D grids only); first: F^k = F^n,
// the pass also writes C
hipError_t ksb_pass(const KsbDev& K, bool first, hipStream_t st);

hipError_t ksb_finalize(const KsbFin& F, hipStream_t st);
// interior of six field components (B then E) times f[c % 3]
hipError_t scale_fields(const GridDev& G, float* const* F, const float f[3], hipStream_t st);
constexpr int kKsbFinBlocks = 512;  // workgroups per box of the finalize copy (grid stride)
hipError_t zero_floats(float* p, int64_t n, hipStream_t st);
hipError_t interior_copy(const GridDev& G, float* guarded, float* dense, int to_dense,
                         hipStream_t st);
hipError_t field_energy(const GridDev& G, float* const* comps, int ncomp, double* part, int nblk,
                        double* out, hipStream_t st);
hipError_t particle_sums(const int32_t* cell, const float* ux, const float* uy, const float* uz,
                         const int32_t* n_live, double* part, int nblk, double* out, hipStream_t st);
constexpr int kPartSums = 7;       // particle_sums rows: gamma-1, u (3), u_c^2/gamma (3)
constexpr int kHistMaxBins = 4096;  // energy_histogram
hipError_t energy_histogram(const int32_t* cell, const float* ux, const float* uy, const float* uz,
                            const int32_t* n_live, const double* edges, int nbins,
                            unsigned long long* counts, int nblk, hipStream_t st);

// Static device scratch of the entry points that allocate nothing (noalloc.hip): the current
// device's copy of one file-scope array of kStaticScratchBytes, its address taken once per
// device.  The histogram variant keeps its edges (FP64, kHistMaxBins + 1) at the start and its
// counts (uint64, kHistMaxBins + 2) at kStaticHistCountsOffset.
constexpr size_t kStaticHistCountsOffset = ((size_t)(kHistMaxBins + 1) * 8 + 255) & ~(size_t)255;
constexpr size_t kStaticScratchBytes =
    (kStaticHistCountsOffset + (size_t)(kHistMaxBins + 2) * 8 + 255) & ~(size_t)255;
hipError_t static_scratch(void** ptr, size_t* bytes);

hipError_t cells_linear_to_packed(const int32_t* lin, int32_t* packed, int64_t n, const int nn[3],
                                  CellCode cc, uint32_t* err, hipStream_t st);
hipError_t cells_packed_to_linear(const int32_t* packed, int32_t* lin, int64_t n, const int nn[3],
                                  CellCode cc, hipStream_t st);
hipError_t device_copy16(void* dst, const void* src, int64_t nwords, hipStream_t st);
hipError_t iota_u32(uint32_t* p, int64_t n, hipStream_t st);
hipError_t set_i32(int32_t* p, int32_t v, hipStream_t st);

}  // namespace pic
