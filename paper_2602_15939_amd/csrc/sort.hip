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
                                                           uint32_t* __restrict__ vals)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n_upper) return;
    const int nl = *n_live;
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

__global__ __launch_bounds__(kBlock) void radix_hist_kernel(const uint32_t* __restrict__ keys,
                                                            int n, int shift,
                                                            uint32_t* __restrict__ hist)
{
    __shared__ uint32_t cnt[256];
    const int tid = threadIdx.x;
    cnt[tid] = 0;
    __syncthreads();
    const int base = blockIdx.x * kChunk;
#pragma unroll 4
    for (int r = 0; r < kItems; r++) {
        const int i = base + r * kBlock + tid;
        if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[tid * gridDim.x + blockIdx.x] = cnt[tid];
}

__global__ __launch_bounds__(kBlock) void radix_scatter_kernel(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin, int n, int shift,
    const uint32_t* __restrict__ hscan, uint32_t* __restrict__ kout, uint32_t* __restrict__ vout)
{
    __shared__ uint32_t base[256];
    __shared__ uint32_t wcnt[4][256];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int nblk = gridDim.x, b = blockIdx.x;
    base[tid] = hscan[tid * nblk + b];
    const unsigned long long lt = (1ull << lane) - 1ull;
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

// off[t] = first sorted position with key >= t, t in [0, n_tiles+1]; off[n_tiles] is the live
// count (dead bin starts there), off[n_tiles+1] = n.
__global__ __launch_bounds__(kBlock) void offsets_kernel(const uint32_t* __restrict__ keys, int n,
                                                         int n_tiles, int32_t* __restrict__ off,
                                                         int32_t* __restrict__ n_live)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (n == 0) {
        if (i <= n_tiles + 1) off[i] = 0;
        if (i == 0) *n_live = 0;
        return;
    }
    if (i >= n) return;
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
                                                             int n, uint32_t* bsum)
{
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
                                                          const uint32_t* bpre)
{
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

hipError_t scan_exclusive(const uint32_t* in, uint32_t* out, int n, uint32_t* scratch,
                          hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int nblk = (n + kChunk - 1) / kChunk;
    uint32_t* bsum = scratch;
    uint32_t* bpre = scratch + nblk;
    scan_blocks_kernel<<<nblk, kBlock, 0, st>>>(in, out, n, nblk > 1 ? bsum : nullptr);
    if (nblk > 1) {
        hipError_t e = scan_exclusive(bsum, bpre, nblk, scratch + 2 * nblk + 64, st);
        if (e != hipSuccess) return e;
        scan_add_kernel<<<nblk, kBlock, 0, st>>>(out, n, bpre);
    }
    return hipGetLastError();
}

size_t sort_hist_words(int64_t n) { return 256 * (size_t)((n + kChunk - 1) / kChunk) + 64; }

// Stable sort by tile; returns the buffer index (0/1) holding the sorted (key, index) pairs.
hipError_t tile_sort(const int32_t* cell, const int32_t* n_live_in, int n_upper, CellCode cc,
                     Tiles tl, SortBufs& sb, int32_t* toff, int32_t* n_live_out, int& which,
                     hipStream_t st)
{
    which = 0;
    if (n_upper > 0) {
        make_keys_kernel<<<(n_upper + kBlock - 1) / kBlock, kBlock, 0, st>>>(
            cell, n_live_in, n_upper, cc, tl, sb.keys[0], sb.vals[0]);
        int bits = 0;
        while ((1u << bits) <= (unsigned)tl.n_tiles) bits++;
        const int passes = (bits + 7) / 8;
        const int nblk = (n_upper + kChunk - 1) / kChunk;
        for (int p = 0; p < passes; p++) {
            const int shift = 8 * p;
            radix_hist_kernel<<<nblk, kBlock, 0, st>>>(sb.keys[which], n_upper, shift, sb.hist);
            hipError_t e = scan_exclusive(sb.hist, sb.hist, 256 * nblk, sb.scratch, st);
            if (e != hipSuccess) return e;
            radix_scatter_kernel<<<nblk, kBlock, 0, st>>>(sb.keys[which], sb.vals[which], n_upper,
                                                          shift, sb.hist, sb.keys[which ^ 1],
                                                          sb.vals[which ^ 1]);
            which ^= 1;
        }
    }
    const int g = ((n_upper > tl.n_tiles + 2 ? n_upper : tl.n_tiles + 2) + kBlock - 1) / kBlock;
    offsets_kernel<<<g, kBlock, 0, st>>>(sb.keys[which], n_upper, tl.n_tiles, toff, n_live_out);
    return hipGetLastError();
}

}  // namespace pic
