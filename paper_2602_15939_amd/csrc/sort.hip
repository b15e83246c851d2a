// sort.hip — stable tile counting sort of the particle arrays (gfx950).
//
// key = tile of the particle's cell (dead particles and slots beyond the live count go to a
// dead bin = n_tiles).  The sort is a stable LSD radix sort of (key, index) pairs with 8-bit
// digits: per-chunk digit histograms, one exclusive scan in digit-major order, and a stable
// scatter that ranks equal digits inside a wave with 8 ballots and a popcount.  The sorted
// indices are the permutation the push kernel reads its particles through, so the particle
// payload itself is moved only once, by the push.  Tile offsets come from the sorted keys.
#include "pic_internal.h"

namespace pic {

constexpr int kItems = 16;                // items per thread per chunk
constexpr int kChunk = kBlock * kItems;   // 4096 items per block


__global__ __launch_bounds__(kBlock) void make_keys_kernel(const int32_t* __restrict__ cell,
                                                           const int32_t* __restrict__ n_live,
                                                           int n_upper, CellCode cc, Tiles tl,
                                                           uint32_t* __restrict__ keys,
                                                           uint32_t* __restrict__ vals, Gate g)
{
    if (g.off()) return;
    const int nl = *n_live;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n_upper; i += gridDim.x * kBlock) {
        uint32_t k = (uint32_t)tl.n_tiles;
        if (i < nl) {
            const int32_t c = cell[i];
            if (c >= 0) {
                int x, y, z;
                cc.decode(c, x, y, z);
                k = (uint32_t)tl.key(x, y, z);
            }
        }
        keys[i] = k;
        vals[i] = (uint32_t)i;
    }
}

// chunks of kChunk keys, a grid-stride loop over them (the grid is capped so that a gated-off
// launch costs a few microseconds)
__global__ __launch_bounds__(kBlock) void radix_hist_kernel(const uint32_t* __restrict__ keys,
                                                            int n, int nchunks, int shift,
                                                            uint32_t* __restrict__ hist, Gate g)
{
    if (g.off()) return;
    __shared__ uint32_t cnt[256];
    const int tid = threadIdx.x;
    for (int ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        cnt[tid] = 0;
        __syncthreads();
        const int base = ch * kChunk;
#pragma unroll 4
        for (int r = 0; r < kItems; r++) {
            const int i = base + r * kBlock + tid;
            if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & 255u], 1u);
        }
        __syncthreads();
        hist[tid * nchunks + ch] = cnt[tid];
        __syncthreads();
    }
}

__global__ __launch_bounds__(kBlock) void radix_scatter_kernel(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin, int n, int nchunks,
    int shift, const uint32_t* __restrict__ hscan, uint32_t* __restrict__ kout,
    uint32_t* __restrict__ vout, Gate g)
{
    if (g.off()) return;
    __shared__ uint32_t base[256];
    __shared__ uint32_t wcnt[4][256];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const unsigned long long lt = (1ull << lane) - 1ull;
    for (int b = blockIdx.x; b < nchunks; b += gridDim.x) {
        base[tid] = hscan[tid * nchunks + b];
        for (int r = 0; r < kItems; r++) {
            wcnt[0][tid] = wcnt[1][tid] = wcnt[2][tid] = wcnt[3][tid] = 0;
            __syncthreads();
            const int i = b * kChunk + r * kBlock + tid;
            const bool valid = i < n;
            const uint32_t key = valid ? kin[i] : 0u;
            const uint32_t val = valid ? vin[i] : 0u;
            const uint32_t d = (key >> shift) & 255u;
            unsigned long long m = __ballot(valid);
#pragma unroll
            for (int bit = 0; bit < 8; bit++) {
                const bool on = (d >> bit) & 1u;
                const unsigned long long bb = __ballot(on);
                m &= on ? bb : ~bb;
            }
            const int rank = __popcll(m & lt);
            if (valid && rank == 0) wcnt[w][d] = (uint32_t)__popcll(m);
            __syncthreads();
            if (valid) {
                uint32_t pre = 0;
                for (int k = 0; k < w; k++) pre += wcnt[k][d];
                const uint32_t pos = base[d] + pre + (uint32_t)rank;
                kout[pos] = key;
                vout[pos] = val;
            }
            __syncthreads();
            base[tid] += wcnt[0][tid] + wcnt[1][tid] + wcnt[2][tid] + wcnt[3][tid];
            __syncthreads();
        }
    }
}

// off[t] = first sorted position with key >= t, t in [0, n_tiles+1]; off[n_tiles] is the live
// count (dead bin starts there), off[n_tiles+1] = n.
__global__ __launch_bounds__(kBlock) void offsets_kernel(const uint32_t* __restrict__ keys, int n,
                                                         int n_tiles, int32_t* __restrict__ off,
                                                         int32_t* __restrict__ n_live, Gate g)
{
    if (g.off()) return;
    const int stride = gridDim.x * kBlock;
    if (n == 0) {
        for (int i = blockIdx.x * kBlock + threadIdx.x; i <= n_tiles + 1; i += stride) off[i] = 0;
        if (blockIdx.x == 0 && threadIdx.x == 0) *n_live = 0;
        return;
    }
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        const int k = (int)keys[i];
        const int kp = i > 0 ? (int)keys[i - 1] : -1;
        for (int t = kp + 1; t <= k; t++) {
            off[t] = i;
            if (t == n_tiles) *n_live = i;
        }
        if (i == n - 1) {
            for (int t = k + 1; t <= n_tiles + 1; t++) {
                off[t] = n;
                if (t == n_tiles) *n_live = n;
            }
        }
    }
}

// ------------------------------------------------------------------ exclusive scan (uint32)
__device__ inline uint32_t wave_incl_scan(uint32_t v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

__global__ __launch_bounds__(kBlock) void scan_blocks_kernel(const uint32_t* in, uint32_t* out,
                                                             int n, uint32_t* bsum, Gate g)
{
    if (g.off()) return;
    __shared__ uint32_t s[kChunk];
    __shared__ uint32_t ws[4];
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kChunk;
    for (int k = 0; k < kItems; k++) {
        const int e = k * kBlock + tid;
        s[e] = base + e < n ? in[base + e] : 0u;
    }
    __syncthreads();
    uint32_t loc[kItems];
    uint32_t sum = 0;
#pragma unroll
    for (int j = 0; j < kItems; j++) {
        loc[j] = s[tid * kItems + j];
        sum += loc[j];
    }
    const uint32_t inc = wave_incl_scan(sum);
    const int w = tid >> 6, lane = tid & 63;
    if (lane == 63) ws[w] = inc;
    __syncthreads();
    uint32_t run = inc - sum;
    for (int k = 0; k < w; k++) run += ws[k];
    const uint32_t tot = ws[0] + ws[1] + ws[2] + ws[3];
#pragma unroll
    for (int j = 0; j < kItems; j++) {
        s[tid * kItems + j] = run;
        run += loc[j];
    }
    __syncthreads();
    for (int k = 0; k < kItems; k++) {
        const int e = k * kBlock + tid;
        if (base + e < n) out[base + e] = s[e];
    }
    if (tid == 0 && bsum) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kBlock) void scan_add_kernel(uint32_t* out, int n,
                                                          const uint32_t* bpre, Gate g)
{
    if (g.off()) return;
    const int64_t i = (int64_t)blockIdx.x * kChunk;
    const uint32_t add = bpre[blockIdx.x];
    for (int k = 0; k < kItems; k++) {
        const int64_t e = i + k * kBlock + threadIdx.x;
        if (e < n) out[e] += add;
    }
}

// words of scratch the scan of n items needs
size_t scan_scratch_words(int64_t n)
{
    size_t w = 0;
    while (n > 1) {
        n = (n + kChunk - 1) / kChunk;
        w += 2 * (size_t)n + 64;
    }
    return w + 64;
}

static hipError_t scan_exclusive(const uint32_t* in, uint32_t* out, int n, uint32_t* scratch,
                                 hipStream_t st, Gate g)
{
    if (n <= 0) return hipSuccess;
    const int nblk = (n + kChunk - 1) / kChunk;
    uint32_t* bsum = scratch;
    uint32_t* bpre = scratch + nblk;
    scan_blocks_kernel<<<nblk, kBlock, 0, st>>>(in, out, n, nblk > 1 ? bsum : nullptr, g);
    if (nblk > 1) {
        hipError_t e = scan_exclusive(bsum, bpre, nblk, scratch + 2 * nblk + 64, st, g);
        if (e != hipSuccess) return e;
        scan_add_kernel<<<nblk, kBlock, 0, st>>>(out, n, bpre, g);
    }
    return hipGetLastError();
}

size_t sort_hist_words(int64_t n) { return 256 * (size_t)((n + kChunk - 1) / kChunk) + 64; }

// grid of the radix kernels: enough workgroups to fill the chip, loops beyond
static unsigned grid_cap(int blocks) { return (unsigned)(blocks < 4096 ? (blocks > 0 ? blocks : 1) : 4096); }

static int radix_passes(const Tiles& tl)
{
    int bits = 0;
    while ((1u << bits) <= (unsigned)tl.n_tiles) bits++;
    return (bits + 7) / 8;
}

static hipError_t radix_tile_sort(const int32_t* cell, const int32_t* n_live_in, int n_upper,
                                  CellCode cc, Tiles tl, SortBufs& sb, int32_t* toff,
                                  int32_t* n_live_out, int& which, hipStream_t st, Gate g)
{
    which = 0;
    if (n_upper > 0) {
        make_keys_kernel<<<grid_cap((n_upper + kBlock - 1) / kBlock), kBlock, 0, st>>>(
            cell, n_live_in, n_upper, cc, tl, sb.keys[0], sb.vals[0], g);
        const int passes = radix_passes(tl);
        const int nchunks = (n_upper + kChunk - 1) / kChunk;
        for (int p = 0; p < passes; p++) {
            const int shift = 8 * p;
            radix_hist_kernel<<<grid_cap(nchunks), kBlock, 0, st>>>(sb.keys[which], n_upper,
                                                                     nchunks, shift, sb.hist, g);
            hipError_t e = scan_exclusive(sb.hist, sb.hist, 256 * nchunks, sb.scratch, st, g);
            if (e != hipSuccess) return e;
            radix_scatter_kernel<<<grid_cap(nchunks), kBlock, 0, st>>>(
                sb.keys[which], sb.vals[which], n_upper, nchunks, shift, sb.hist,
                sb.keys[which ^ 1], sb.vals[which ^ 1], g);
            which ^= 1;
        }
    }
    const int nb = ((n_upper > tl.n_tiles + 2 ? n_upper : tl.n_tiles + 2) + kBlock - 1) / kBlock;
    offsets_kernel<<<grid_cap(nb), kBlock, 0, st>>>(sb.keys[which], n_upper, tl.n_tiles, toff,
                                                    n_live_out, g);
    return hipGetLastError();
}

// Stable sort by tile; returns the buffer index (0/1) holding the sorted (key, index) pairs.
hipError_t tile_sort(const int32_t* cell, const int32_t* n_live_in, int n_upper, CellCode cc,
                     Tiles tl, SortBufs& sb, int32_t* toff, int32_t* n_live_out, int& which,
                     hipStream_t st)
{
    return radix_tile_sort(cell, n_live_in, n_upper, cc, tl, sb, toff, n_live_out, which, st,
                           Gate{nullptr, 0});
}

// ------------------------------------------------------------------ migration sort
// Between two sorts a particle moves less than one cell, so the particles of source tile s
// (the slots toff_prev[s] .. toff_prev[s+1]-1, in the order of the previous sort) land in s or
// one of its neighbours.  The stable counting sort by the new tile then needs, per source tile,
// only the counts per direction (kMigDirs of them) instead of a full radix sort:
//   count:   per source tile, particles per direction;
//   offsets: per destination tile, its (at most 27) sources in increasing tile order give each
//            (source, direction) pair its offset inside the destination, and the total;
//   scans:   destination starts (= the new tile offsets) and the dead bin's per-source starts;
//   scatter: per source tile, in slot order, stable ranks per direction by wave ballots.
// The result equals the stable radix sort: within a destination tile the particles come in
// increasing source tile, i.e. increasing slot, for the live slots (the permutation's
// observable part).  Slots from the previous dead bin stay dead at the end, after the
// particles that died since.

__device__ inline void dir_steps(int d, int& dx, int& dy, int& dz)
{
    dx = d % 3 - 1;
    dy = (d / 3) % 3 - 1;
    dz = d / 9 - 1;
}

__device__ inline bool dir_possible(const MigGeo& g, int dx, int dy, int dz)
{
    return (g.nt[0] > 1 || dx == 0) && (g.nt[1] > 1 || dy == 0) && (g.nt[2] > 1 || dz == 0);
}

__device__ inline int wrap_tile(int v, int n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

// tile reached from source (sx, sy, sz) in direction (dx, dy, dz)
__device__ inline int mig_dst(const MigGeo& g, int sx, int sy, int sz, int dx, int dy, int dz)
{
    int tx = sx + dx, wx = 0;
    if (tx >= g.nt[0]) {
        tx -= g.nt[0];
        wx = 1;
    } else if (tx < 0) {
        tx += g.nt[0];
        wx = -1;
    }
    const int shift = wx > 0 ? g.cy_out : (wx < 0 ? g.cy_in : 0);
    return tx + g.nt[0] * (wrap_tile(sy + dy + shift, g.nt[1]) + g.nt[1] * wrap_tile(sz + dz, g.nt[2]));
}

// source tile that reaches (tx, ty, tz) in direction (dx, dy, dz)
__device__ inline int mig_src(const MigGeo& g, int tx, int ty, int tz, int dx, int dy, int dz)
{
    int sx = tx - dx, wx = 0;
    if (sx < 0) {  // the source sits at the outer end and left through the outer face
        sx += g.nt[0];
        wx = 1;
    } else if (sx >= g.nt[0]) {
        sx -= g.nt[0];
        wx = -1;
    }
    const int shift = wx > 0 ? g.cy_out : (wx < 0 ? g.cy_in : 0);
    return sx + g.nt[0] * (wrap_tile(ty - dy - shift, g.nt[1]) + g.nt[1] * wrap_tile(tz - dz, g.nt[2]));
}

constexpr int kMigItems = 4;  // particles per thread per round of the migration kernels

__device__ __attribute__((always_inline)) inline void mig_count_body(const MigCountArgs& a, int blk, int, int)
{
    const int32_t* __restrict__ cell = a.cell;
    const int32_t* __restrict__ toff_prev = a.toff_prev;
    const CellCode& cc = a.cc;
    const MigGeo& g = a.g;
    __shared__ uint32_t cnt[kMigDirs];
    const int s = blk, tid = threadIdx.x;
    if (tid < kMigDirs) cnt[tid] = 0;
    __syncthreads();
    int sx, sy, sz;
    tile_coords(g, s, sx, sy, sz);
    const int beg = toff_prev[s], end = toff_prev[s + 1];
    uint32_t stay = 0;
    bool bad = false;
    for (int cb = beg; cb < end; cb += kBlock * kMigItems) {
        int32_t c[kMigItems];
#pragma unroll
        for (int j = 0; j < kMigItems; j++) {
            const int i = cb + j * kBlock + tid;
            c[j] = i < end ? cell[i] : INT32_MIN;
        }
#pragma unroll
        for (int j = 0; j < kMigItems; j++) {
            if (c[j] == INT32_MIN) continue;
            const int d = mig_dir(g, cc, sx, sy, sz, c[j]);
            if (d == 13)
                stay++;
            else if (d >= 0)
                atomicAdd(&cnt[d], 1u);
            else
                bad = true;
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) stay += __shfl_xor(stay, o, 64);
    if ((tid & 63) == 0 && stay) atomicAdd(&cnt[13], stay);
    if (bad) {
        *a.fallback = 1;
        if (a.err) atomicOr(a.err, kErrSort);
    }
    __syncthreads();
    if (tid < kMigDirs) a.mcnt[(size_t)s * kMigDirs + tid] = cnt[tid];
}
PIC_BATCHED_KERNEL(mig_count, MigCountArgs, kBlock)

// one wave per destination tile
__device__ __attribute__((always_inline)) inline void mig_offsets_body(const MigOffArgs& a, int blk, int, int)
{
    if (a.gate.off()) return;
    const uint32_t* __restrict__ mcnt = a.mcnt;
    const MigGeo& g = a.g;
    uint32_t* __restrict__ mpre = a.mpre;
    uint32_t* __restrict__ tot = a.tot;
    uint32_t* __restrict__ dcnt = a.dcnt;
    const int lane = threadIdx.x & 63;
    const int t = blk * (kBlock / 64) + (threadIdx.x >> 6);
    if (t == 0 && lane == 0) {
        tot[g.n_tiles] = 0;
        dcnt[g.n_tiles] = 0;
    }
    if (t >= g.n_tiles) return;
    int tx, ty, tz;
    tile_coords(g, t, tx, ty, tz);
    uint32_t c = 0;
    int key = 0x7fffffff, src = 0;
    if (lane < 27) {
        int dx, dy, dz;
        dir_steps(lane, dx, dy, dz);
        if (dir_possible(g, dx, dy, dz)) {
            src = mig_src(g, tx, ty, tz, dx, dy, dz);
            key = src;
            c = mcnt[(size_t)src * kMigDirs + lane];
        }
    }
    uint32_t pre = 0, total = 0;
    for (int k = 0; k < 27; k++) {
        const int kk = __shfl(key, k, 64);
        const uint32_t ck = __shfl(c, k, 64);
        total += ck;
        if (kk < key) pre += ck;
    }
    if (lane < 27 && key != 0x7fffffff) mpre[(size_t)src * kMigDirs + lane] = pre;
    if (lane == 0) {
        tot[t] = total;
        dcnt[t] = mcnt[(size_t)t * kMigDirs + kMigDead];
    }
}
PIC_BATCHED_KERNEL(mig_offsets, MigOffArgs, kBlock)

// block s < n_tiles: the particles of source tile s (the newly dead go to the dead bin after
// the live ones); block n_tiles: the offsets of the dead bin and the live count
__device__ __attribute__((always_inline)) inline void mig_scatter_body(const MigScatterArgs& a, int blk, int, int)
{
    if (a.gate.off()) return;
    const int32_t* __restrict__ cell = a.cell;
    const int32_t* __restrict__ toff_prev = a.toff_prev;
    const int n_upper = a.n_upper;
    const CellCode& cc = a.cc;
    const MigGeo& g = a.g;
    const uint32_t* __restrict__ mpre = a.mpre;
    const uint32_t* __restrict__ start = a.start;
    const uint32_t* __restrict__ dpre = a.dpre;
    uint32_t* __restrict__ perm = a.perm;
    int32_t* __restrict__ toff = a.toff;
    int32_t* __restrict__ n_live = a.n_live;
    __shared__ uint32_t run[2][kMigDirs];
    __shared__ uint32_t wc[kMigItems][kBlock / 64][kMigDirs];   // per (item, wave): count per direction
    __shared__ uint32_t pre[kMigItems][kBlock / 64][kMigDirs];  // exclusive prefix over (item, wave)
    const int s = blk, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint32_t live = start[g.n_tiles];
    if (s == g.n_tiles) {
        // the slots of the previous dead bin stay dead at the end; nothing reads the
        // permutation past the live count, so they are not enumerated again
        if (tid == 0) {
            toff[g.n_tiles] = (int32_t)live;
            toff[g.n_tiles + 1] = n_upper;
            *n_live = (int32_t)live;
        }
        return;
    }
    int sx, sy, sz;
    tile_coords(g, s, sx, sy, sz);
    if (tid == 0) toff[s] = (int32_t)start[s];
    if (tid < kMigDirs) {
        uint32_t b = 0;
        if (tid == kMigDead) {
            b = live + dpre[s];
        } else {
            int dx, dy, dz;
            dir_steps(tid, dx, dy, dz);
            if (dir_possible(g, dx, dy, dz))
                b = start[mig_dst(g, sx, sy, sz, dx, dy, dz)] + mpre[(size_t)s * kMigDirs + tid];
        }
        run[0][tid] = b;
    }
    __syncthreads();
    const int beg = toff_prev[s], end = toff_prev[s + 1];
    const unsigned long long lt = (1ull << lane) - 1ull;
    int p = 0;
    // rounds of kBlock * kMigItems slots; item j of a round covers slots j*kBlock .. +kBlock-1,
    // so the stable order inside a round is (item, wave, lane)
    for (int cb = beg; cb < end; cb += kBlock * kMigItems) {
        int32_t c[kMigItems];
#pragma unroll
        for (int j = 0; j < kMigItems; j++) {
            const int i = cb + j * kBlock + tid;
            c[j] = i < end ? cell[i] : 0;
        }
        int d[kMigItems];
        uint32_t rank[kMigItems];
#pragma unroll
        for (int j = 0; j < kMigItems; j++) {
            const bool valid = cb + j * kBlock + tid < end;
            d[j] = valid ? mig_dir(g, cc, sx, sy, sz, c[j]) : -1;
            // lanes with the same key (direction + 1, 5 bits; 0 = none): the AND over the key
            // bits of the ballot of that bit or of its complement
            const uint32_t key = (uint32_t)(d[j] + 1);
            unsigned long long same = ~0ull;
#pragma unroll
            for (int bit = 0; bit < 5; bit++) {
                const unsigned long long m = __ballot((key >> bit) & 1u);
                same &= ((key >> bit) & 1u) ? m : ~m;
            }
            rank[j] = (uint32_t)__popcll(same & lt);
            if (lane < kMigDirs) wc[j][w][lane] = 0u;
            // the lowest lane of each group writes the group's count (same wave: in order)
            if (d[j] >= 0 && rank[j] == 0) wc[j][w][d[j]] = (uint32_t)__popcll(same);
        }
        __syncthreads();
        // per direction, the exclusive prefix over (item, wave) and the running offset
        if (tid < kMigDirs) {
            uint32_t a = run[p][tid];
#pragma unroll
            for (int jj = 0; jj < kMigItems; jj++)
#pragma unroll
                for (int k = 0; k < kBlock / 64; k++) {
                    pre[jj][k][tid] = a;
                    a += wc[jj][k][tid];
                }
            run[p ^ 1][tid] = a;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kMigItems; j++)
            if (d[j] >= 0) perm[pre[j][w][d[j]] + rank[j]] = (uint32_t)(cb + j * kBlock + tid);
        p ^= 1;
    }
}
PIC_BATCHED_KERNEL(mig_scatter, MigScatterArgs, kBlock)

// Exclusive scan of n words by one workgroup (the per-tile arrays of a small box).
__device__ __attribute__((always_inline)) inline void scan_small_body(const ScanArgs& a, int, int, int)
{
    if (a.gate.off()) return;
    __shared__ uint32_t ws[kBlock / 64];
    __shared__ uint32_t carry;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (tid == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < a.n; base += kBlock) {
        const int i = base + tid;
        const uint32_t v = i < a.n ? a.in[i] : 0u;
        uint32_t inc = v;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t t = __shfl_up(inc, o, 64);
            if (lane >= o) inc += t;
        }
        if (lane == 63) ws[w] = inc;
        __syncthreads();
        uint32_t pre = carry;
        for (int k = 0; k < w; k++) pre += ws[k];
        if (i < a.n) a.out[i] = pre + inc - v;
        __syncthreads();
        if (tid == kBlock - 1) carry = pre + inc;
        __syncthreads();
    }
}
PIC_BATCHED_KERNEL(scan_small, ScanArgs, kBlock)

// the box's count of radix fallbacks (the sorts of two species may add at the same time)
__global__ void count_fallback_kernel(unsigned long long* ctr, Gate g)
{
    if (!g.off()) atomicAdd(ctr, 1ull);
}

hipError_t sort_batch(SortBatchKind k, const void* table, UnitMap m, int blocks, hipStream_t st)
{
    if (blocks <= 0) return hipSuccess;
    switch (k) {
    case kBatchMigCount:
        mig_count_batch<<<blocks, kBlock, 0, st>>>(static_cast<const MigCountArgs*>(table), m);
        break;
    case kBatchMigOffsets:
        mig_offsets_batch<<<blocks, kBlock, 0, st>>>(static_cast<const MigOffArgs*>(table), m);
        break;
    case kBatchScan: scan_small_batch<<<blocks, kBlock, 0, st>>>(static_cast<const ScanArgs*>(table), m); break;
    case kBatchMigScatter:
        mig_scatter_batch<<<blocks, kBlock, 0, st>>>(static_cast<const MigScatterArgs*>(table), m);
        break;
    }
    return hipGetLastError();
}

int sort_result_buffer(const Tiles& tl) { return radix_passes(tl) & 1; }

size_t migrate_scratch_words(int n_tiles) { return scan_scratch_words((int64_t)n_tiles + 1); }

hipError_t migrate_sort(const int32_t* cell, const int32_t* toff_prev, int n_upper, CellCode cc,
                        Tiles tl, const MigGeo& mg, SortBufs& sb, int32_t* toff,
                        int32_t* n_live_out, int& which, unsigned long long* n_fallback,
                        bool counts_ready, hipStream_t st)
{
    const int nt = tl.n_tiles;
    const Gate mig{sb.fallback, 0}, radix{sb.fallback, 1};
    which = radix_passes(tl) & 1;  // where the radix fallback leaves its result
    if (!counts_ready) {
        if (set_i32(sb.fallback, 0, st) != hipSuccess) return hipGetLastError();
        mig_count_kernel<<<nt, kBlock, 0, st>>>(
            MigCountArgs{cell, toff_prev, cc, mg, sb.mcnt, sb.fallback, nullptr});
    }
    mig_offsets_kernel<<<(nt + kBlock / 64 - 1) / (kBlock / 64), kBlock, 0, st>>>(
        MigOffArgs{sb.mcnt, mg, sb.mpre, sb.tot, sb.dcnt, mig});
    hipError_t e = scan_exclusive(sb.tot, sb.start, nt + 1, sb.mscratch, st, mig);
    if (e == hipSuccess) e = scan_exclusive(sb.dcnt, sb.dpre, nt + 1, sb.mscratch, st, mig);
    if (e != hipSuccess) return e;
    mig_scatter_kernel<<<nt + 1, kBlock, 0, st>>>(
        MigScatterArgs{cell, toff_prev, n_upper, cc, mg, sb.mpre, sb.start, sb.dpre, sb.vals[which],
                       toff, n_live_out, mig});
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    int w2 = 0;
    e = radix_tile_sort(cell, toff_prev + nt, n_upper, cc, tl, sb, toff, n_live_out, w2, st, radix);
    if (e == hipSuccess) count_fallback_kernel<<<1, 1, 0, st>>>(n_fallback, radix);
    return e == hipSuccess ? hipGetLastError() : e;
}

}  // namespace pic
