// api.cpp — host driver of the C ABI declared in include/pic.h: box lifetime, state
// transfer, per-step scalars (computed in FP64 on the host: t, Delta y_s(t), l(t), Lambda)
// and the orchestration of the HIP kernels on the box stream.
#include "pic.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <new>
#include <tuple>
#include <vector>

#include "pic_internal.h"

using namespace pic;

namespace {

constexpr double kPi = 3.14159265358979323846;

struct Species {
    int64_t cap = 0;
    int n_upper = 0;  // slots the sort looks at (host upper bound of the live count)
    int cur = 0;      // particle buffer holding the current state
    int32_t* cell[2] = {};
    float* off[2][3] = {};
    float* u[2][3] = {};
    uint32_t* id[2] = {};
    float* dr[2][3] = {};
    SortBufs sb{};
    int which = 0;          // sort buffer holding the sorted (key, index) pairs
    int32_t* toff[2] = {};  // tile offsets (n_tiles + 2) of the last two sorts
    int toff_cur = 0;       // toff[toff_cur] belongs to the last sort
    bool grouped = false;   // particle arrays are in the slot order of toff[toff_cur] (a push ran)
    bool counts_ready = false;  // that push also wrote the migration counts of the next sort
    int32_t* n_live = nullptr;
    int32_t* ws_cell = nullptr;
    float* ws_off[3] = {};
    float* ws_disp[3] = {};
    double qm = 0, q = 0;
};

// Staging of the descriptor tables of batched steps (two buffers, alternating) and the
// executable graphs captured over them.  A library-owned box grows its own on demand; a
// caller-owned one (pic_batch) has fixed buffers the caller allocated.
struct Stager {
    struct Buf {
        void* host = nullptr;  // pinned
        void* dev = nullptr;
        size_t cap = 0;
        hipEvent_t copied = nullptr;  // the last transfer out of host has completed
    } buf[2];
    int cur = 0;
    bool caller = false;  // buffers owned by the caller: never reallocated
    // executable graphs keyed by the box set, the staging buffer and the launch sequence (grid
    // sizes and table offsets); least recently used last
    struct StepGraph {
        std::vector<uint64_t> key;
        hipGraphExec_t exec = nullptr;
    };
    std::vector<StepGraph> graphs;
};

// Device and pinned host memory the library holds (library-owned boxes, their unfused-deposit
// workspaces and batched-step staging); a box created on caller memory adds nothing.
std::atomic<int64_t> g_dev_bytes{0}, g_host_bytes{0};

hipError_t lib_malloc(void** p, size_t bytes)
{
    const hipError_t e = hipMalloc(p, bytes);
    if (e == hipSuccess) g_dev_bytes += (int64_t)bytes;
    return e;
}
void lib_free(void* p, size_t bytes)
{
    if (!p) return;
    hipFree(p);
    g_dev_bytes -= (int64_t)bytes;
}
hipError_t lib_host_malloc(void** p, size_t bytes)
{
    const hipError_t e = hipHostMalloc(p, bytes);
    if (e == hipSuccess) g_host_bytes += (int64_t)bytes;
    return e;
}
void lib_host_free(void* p, size_t bytes)
{
    if (!p) return;
    hipHostFree(p);
    g_host_bytes -= (int64_t)bytes;
}

void stager_release(Stager& sg)
{
    for (auto& g : sg.graphs) hipGraphExecDestroy(g.exec);
    sg.graphs.clear();
    for (auto& b : sg.buf) {
        if (!sg.caller) {
            lib_host_free(b.host, b.cap);
            lib_free(b.dev, b.cap);
        }
        if (b.copied) hipEventDestroy(b.copied);
        b = Stager::Buf{};
    }
}

}  // namespace

struct pic_batch {
    Stager sg;
    hipStream_t st = nullptr;
};

struct pic_box {
    pic_box_desc d{};
    hipStream_t st = nullptr;
    int dim = 3;
    int n[3] = {1, 1, 1};
    int tile[3] = {1, 1, 1};
    GridDev G{};
    int64_t comp_elems = 0;  // floats per guarded component array
    int64_t origin = 0;      // offset of interior (0,0,0)
    CellCode cc{};
    Tiles tl{};
    int nsp = 1;
    Species sp[kMaxSpecies];
    MigGeo mg{};            // migration sort geometry (y shifts set by each push)
    bool mig_ok = false;    // the tile grid admits the migration sort
    // field sets: set[s][0..2] = B, set[s][3..5] = E (shearing box keeps 3 sets for the
    // fixed-point iterates); cur_set is the one holding the fields
    float* set[3][6] = {};
    int nsets = 1;
    int cur_set = 0;
    float* J[3] = {};
    float* Jt[3] = {};
    float* J0 = nullptr;  // interior pointer of the first current array's x component
    float* mj = nullptr;
    uint32_t* err = nullptr;
    unsigned long long* ctr = nullptr;
    uint32_t* conv = nullptr;  // shearing box: convergence record of the tolerance-mode sweeps
    int last_sweeps = 0;       // sweeps of the last Maxwell step (-1: the device record has it)
    double* red_part = nullptr;
    double* red_out = nullptr;
    double* hist_edges = nullptr;               // energy histogram: edges ...
    unsigned long long* hist_counts = nullptr;  // ... and counts
    int64_t step = 0;
    int64_t n_migrations = 0;
    // staging and graphs of batched steps led by this box through pic_step (library-owned
    // boxes only; boxes on caller memory step in batches through pic_step_batch)
    Stager stager;
    uint64_t uid = 0;  // unique over the process lifetime (graph keys)
    bool sorted = false;
    bool deposit_pending = false;
    bool record_valid = false;  // the unfused-deposit workspace holds the last push's record
    // PIC_SORT_OVERLAP: the sort of each species on a stream of its own beside the box stream,
    // joined by the next call that touches particles or the sort (default priority, created
    // on first use)
    hipStream_t side[kMaxSpecies] = {};
    hipEvent_t fork_ev = nullptr, side_ev[kMaxSpecies] = {};
    bool side_pending = false;
    bool track_ids = false;
    bool caller_mem = false;  // created on caller memory (pic_box_mem): never allocates
    std::vector<std::pair<void*, size_t>> allocs;
    // pic_box_create takes all of the box's device memory in one allocation: a first pass over
    // the buffer list measures it, a second carves it (from the library's allocation, or from
    // the caller's workspace)
    int alloc_pass = 0;  // 0: separate allocations, 1: measuring, 2: carving
    char* arena = nullptr;
    size_t arena_off = 0;

    float* E(int c) const { return set[cur_set][3 + c]; }
    float* B(int c) const { return set[cur_set][c]; }
};

namespace {

constexpr int kRedBlocks = 1024;
constexpr int kRowAlign = 32;  // floats per 128-byte line

int32_t hip_fail(hipError_t e) { return e == hipSuccess ? PIC_OK : PIC_EDEVICE; }

// make the box stream wait for the sorts queued on the side streams (PIC_SORT_OVERLAP)
int32_t side_join(pic_box* b)
{
    if (!b->side_pending) return PIC_OK;
    b->side_pending = false;
    for (int s = 0; s < b->nsp; s++)
        if (hipStreamWaitEvent(b->st, b->side_ev[s], 0) != hipSuccess) return PIC_EDEVICE;
    return PIC_OK;
}

// the leaky box's escape rule applies: always in the leaky frame, on request in the others
bool escapes(const pic_box_desc* d)
{
    return d->frame == PIC_FRAME_LEAKY || (d->flags & PIC_BOX_ESCAPE) != 0;
}
// frames with the shearing-box geometry (Sec. 2), and with the expanding-box factors (Sec. 3);
// the combined frame has both
bool sheared(const pic_box_desc* d)
{
    return d->frame == PIC_FRAME_SHEAR || d->frame == PIC_FRAME_SHEAR_EXPAND;
}
bool expanding(const pic_box_desc* d)
{
    return d->frame == PIC_FRAME_EXPAND || d->frame == PIC_FRAME_SHEAR_EXPAND;
}

template <class T>
int32_t dalloc(pic_box* b, T*& p, size_t count)
{
    if (count == 0) count = 1;
    const size_t bytes = (count * sizeof(T) + 255) & ~(size_t)255;
    if (b->alloc_pass == 1) {  // measuring
        b->arena_off += bytes;
        p = nullptr;
        return PIC_OK;
    }
    if (b->alloc_pass == 2) {  // carving
        p = reinterpret_cast<T*>(b->arena + b->arena_off);
        b->arena_off += bytes;
        return PIC_OK;
    }
    if (b->caller_mem) return PIC_ESTATE;  // a box on caller memory never allocates
    void* q = nullptr;
    if (lib_malloc(&q, bytes) != hipSuccess) return PIC_ENOMEM;
    b->allocs.push_back({q, bytes});
    p = static_cast<T*>(q);
    return PIC_OK;
}

int ceil_log2(int v)
{
    int b = 0;
    while ((1 << b) < v) b++;
    return b;
}

double time_of(const pic_box* b, int64_t step) { return (double)step * b->d.dt; }

// Sec. 2.1: Delta y_s(t) = s Omega0 (x_o - x_i) t, reduced modulo n[1] (the combined frame
// scales x and y together, so the offset keeps its form in the expanding coordinates)
double shear_offset(const pic_box* b, double t)
{
    if (!sheared(&b->d)) return 0.0;
    const double ny = b->n[1];
    double v = std::fmod(b->d.shear_s * b->d.shear_omega0 * (double)b->n[0] * t, ny);
    if (v < 0) v += ny;
    if (v >= ny) v = 0.0;
    return v;
}

// Sec. 3.1: l_d(t) = 1 + adot t on the expanding axes
double scale_of(const pic_box* b, int axis, double t)
{
    if (!expanding(&b->d) || !((b->d.expand_axis_mask >> axis) & 1)) return 1.0;
    return 1.0 + b->d.expand_adot * t;
}

// ---------------------------------------------------------------- reinjection table
// Maxwell-Juttner inverse CDF of |u| (density u^2 exp(-(gamma-1)/theta)): bulk quantiles
// i/kMjBins and tail quantiles 1 - 2^-(12 + 20 k/kMjTail).  Panel masses by 8-point
// Gauss-Legendre, summed from the top; inside the bracketing panel the quantile is refined by
// Newton iterations on the partial-panel mass.
const double kGLx[4] = {0.1834346424956498, 0.5255324099163290, 0.7966664774136267,
                        0.9602898564975363};
const double kGLw[4] = {0.3626837833783620, 0.3137066458778873, 0.2223810344533745,
                        0.1012285362903763};

double mj_g(double u, double th) { return u * u * std::exp(-(std::sqrt(1.0 + u * u) - 1.0) / th); }

double gl_mass(double a, double c, double th)
{
    const double m = 0.5 * (a + c), h = 0.5 * (c - a);
    double s = 0;
    for (int i = 0; i < 4; i++) s += kGLw[i] * (mj_g(m - h * kGLx[i], th) + mj_g(m + h * kGLx[i], th));
    return s * h;
}

void build_mj_table(double theta, std::vector<float>& out)
{
    const int P = 1 << 15;
    const double gmax = 1.0 + 60.0 * theta, umax = std::sqrt(gmax * gmax - 1.0), h = umax / P;
    std::vector<double> Q(P + 1, 0.0);  // mass above panel edge k
    for (int k = P - 1; k >= 0; k--) Q[k] = Q[k + 1] + gl_mass(k * h, (k + 1) * h, theta);
    const double tot = Q[0];
    auto quantile = [&](double q) -> double {  // |u| with (mass above)/tot = q
        if (q >= 1.0) return 0.0;
        const double target = q * tot;
        int lo = 0, hi = P;  // Q[lo] >= target > Q[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) / 2;
            if (Q[mid] >= target)
                lo = mid;
            else
                hi = mid;
        }
        const double a = lo * h, c = hi * h;
        double u = a + (Q[lo] - target) / (Q[lo] - Q[hi]) * h;
        for (int it = 0; it < 8; it++) {
            const double f = Q[hi] + gl_mass(u, c, theta) - target;
            const double fp = -mj_g(u, theta);
            if (fp == 0.0) break;
            double un = u - f / fp;
            if (un < a) un = a;
            if (un > c) un = c;
            u = un;
        }
        return u;
    };
    out.resize(kMjBins + kMjTail);
    for (int i = 0; i < kMjBins; i++) out[i] = (float)quantile(1.0 - (double)i / kMjBins);
    const int bits = 12;  // log2(kMjBins)
    for (int k = 0; k <= kMjTail; k++)
        out[kMjBins - 1 + k] = (float)quantile(std::ldexp(1.0, -bits) *
                                               std::exp2(-(32.0 - bits) * k / kMjTail));
}

// ---------------------------------------------------------------- descriptor of one push
void set_migration_shift(pic_box* b, int dys_int);

StepDev make_step(pic_box* b)
{
    StepDev P{};
    P.dim = b->dim;
    P.frame = b->d.frame;
    for (int k = 0; k < 3; k++) P.n[k] = b->n[k];
    P.cc = b->cc;
    P.tl = b->tl;
    P.sy = b->G.sy;
    P.sz = b->G.sz;
    for (int c = 0; c < 3; c++) {
        P.E[c] = b->E(c);
        P.B[c] = b->B(c);
        P.J[c] = b->J[c];
    }
    const double dt = b->d.dt;
    P.dt = (float)dt;
    const double tn = time_of(b, b->step), th = tn + 0.5 * dt, t1 = tn + dt;
    const double sO = b->d.shear_s * b->d.shear_omega0;
    P.sO = (float)sO;
    P.om_dt = (float)(b->d.shear_omega0 * dt);
    P.alpha1 = (float)(sO * dt / 2.0);
    P.half_nx = 0.5f * (float)b->n[0];
    const double dys1 = shear_offset(b, t1);
    const double fl = std::floor(dys1);
    P.dys_int = (int)fl;
    P.dys_frac = (float)(dys1 - fl);
    if (P.dys_frac >= 1.f) {  // FP32 rounding of a fraction just below 1
        P.dys_frac = 0.f;
        P.dys_int = (P.dys_int + 1) % b->n[1];
    }
    // the push counts the migration directions of the next sort (its y shifts of the
    // shearing-box x crossings follow this step's Delta y_s)
    set_migration_shift(b, P.dys_int);
    P.count_mig = b->mig_ok ? 1 : 0;
    P.mig_latch = 0;
    P.mg = b->mg;
    for (int s = 0; s < b->nsp; s++) {
        P.mcnt[s] = b->sp[s].sb.mcnt;
        P.mfb[s] = b->sp[s].sb.fallback;
    }
    for (int k = 0; k < 3; k++) {
        const double rate =
            (expanding(&b->d) && ((b->d.expand_axis_mask >> k) & 1)) ? b->d.expand_adot : 0.0;
        const double lam = -0.5 * dt * rate / scale_of(b, k, tn);  // Lambda at t^n
        P.lam1p[k] = (float)(1.0 + lam);
        P.ltil[k] = (float)((1.0 + lam) / (1.0 - lam));
        P.tfac[k] = (float)(1.0 / (1.0 - lam));
        P.linv[k] = (float)(1.0 / scale_of(b, k, th));  // (L^-1)^{n+1/2}
    }
    P.leaky_mode = b->d.leaky_mode;
    P.use_3vec = b->d.leaky_use_3vec;
    P.escape = escapes(&b->d) ? 1 : 0;
    P.l_esc = (float)b->d.leaky_l_esc;
    {
        const double p = b->d.leaky_t_esc > 0 ? dt / b->d.leaky_t_esc : 0.0;
        const double th32 = std::floor(p * 4294967296.0);
        P.esc_thr = th32 >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)th32;
    }
    P.g2thr = b->d.leaky_gamma_thr * b->d.leaky_gamma_thr - 1.0;
    P.key0 = (uint32_t)b->d.seed;
    P.key1 = (uint32_t)(b->d.seed >> 32);
    P.step_lo = (uint32_t)b->step;
    P.box_id = b->d.box_id;
    P.mj = b->mj;
    // Largest single deposit contribution: |q|/dt * |DS| * P with |DS| < 1/2 (CFL), or the 2D
    // J_z term |q v_z W| <= |q|; it maps to 2^30 fixed-point units of the LDS tile sum.
    {
        double qmax = 0.0;
        for (int s = 0; s < b->nsp; s++) qmax = std::fmax(qmax, std::fabs(b->sp[s].q));
        const double bound = std::fmax(0.5 * qmax / dt, qmax);
        const double unit = bound > 0 ? bound / 1073741824.0 : 1.0;
        P.junit = (float)unit;
        P.jscale = (float)(1.0 / unit);
    }
    P.err = b->err;
    P.ctr = b->ctr;
    P.nsp = b->nsp;
    P.track_ids = b->track_ids ? 1 : 0;
    P.count_sl = (b->d.flags & PIC_BOX_COUNT_SUPERLUMINAL) ? 1 : 0;
    for (int s = 0; s < b->nsp; s++) {
        Species& S = b->sp[s];
        SpeciesDev& D = P.sp[s];
        const int i = S.cur, o = S.cur ^ 1;
        D.cell_in = S.cell[i];
        D.cell_out = S.cell[o];
        for (int c = 0; c < 3; c++) {
            D.off_in[c] = S.off[i][c];
            D.off_out[c] = S.off[o][c];
            D.u_in[c] = S.u[i][c];
            D.u_out[c] = S.u[o][c];
            D.dr_in[c] = S.dr[i][c];
            D.dr_out[c] = S.dr[o][c];
            D.ws_off[c] = S.ws_off[c];
            D.ws_disp[c] = S.ws_disp[c];
        }
        D.id_in = S.id[i];
        D.id_out = S.id[o];
        D.perm = reinterpret_cast<const int32_t*>(S.sb.vals[S.which]);
        D.toff = S.toff[S.toff_cur];
        D.ws_cell = S.ws_cell;
        D.qm_hdt = (float)(S.qm * dt / 2.0);
        D.q_dt = (float)(S.q / dt);
    }
    return P;
}

int32_t check_boxes(pic_box* const* boxes, int32_t nb)
{
    if (!boxes || nb < 1) return PIC_EINVAL;
    for (int i = 0; i < nb; i++)
        if (!boxes[i]) return PIC_EINVAL;
    return PIC_OK;
}

// Tile decomposition of the box (power-of-two tile edges); the migration sort applies with whole
// tiles and, on every axis, one tile or at least three (so that the steps -1, 0, +1 reach
// distinct tiles); the shearing box needs the x crossings visible in the tile index.
void set_tiling(pic_box* b, const int tile[3])
{
    for (int k = 0; k < 3; k++) {
        b->tile[k] = tile[k];
        b->tl.lt[k] = ceil_log2(tile[k]);
        b->tl.nt[k] = (b->n[k] + tile[k] - 1) / tile[k];
    }
    b->tl.n_tiles = b->tl.nt[0] * b->tl.nt[1] * b->tl.nt[2];
    b->mig_ok = true;
    for (int k = 0; k < 3; k++) {
        b->mg.nt[k] = b->tl.nt[k];
        b->mg.lt[k] = b->tl.lt[k];
        if (b->n[k] % tile[k] != 0 || b->tl.nt[k] == 2) b->mig_ok = false;
    }
    if (sheared(&b->d) && b->tl.nt[0] < 3) b->mig_ok = false;
    b->mg.n_tiles = b->tl.n_tiles;
}

// the largest tile count over the supported shapes (tile-indexed workspace is sized for it)
int max_tiles(int dim, const int n[3])
{
    int c[8][3];
    const int nc = tile_candidates(dim, false, c, 8);
    int m = 1;
    for (int i = 0; i < nc; i++) {
        int t = 1;
        for (int k = 0; k < 3; k++) t *= (n[k] + c[i][k] - 1) / c[i][k];
        m = std::max(m, t);
    }
    return m;
}

// the tile sort of species s, queued on stream st (the species' buffers only: the sorts of
// different species may run at the same time)
int32_t sort_species(pic_box* b, int s, hipStream_t st)
{
    Species& S = b->sp[s];
    hipError_t e;
    if (b->mig_ok && S.grouped) {
        const int nxt = S.toff_cur ^ 1;
        e = migrate_sort(S.cell[S.cur], S.toff[S.toff_cur], S.n_upper, b->cc, b->tl, b->mg, S.sb,
                         S.toff[nxt], S.n_live, S.which, b->ctr + 2, S.counts_ready, st);
        S.toff_cur = nxt;
        b->n_migrations++;
    } else {
        e = tile_sort(S.cell[S.cur], S.n_live, S.n_upper, b->cc, b->tl, S.sb, S.toff[S.toff_cur],
                      S.n_live, S.which, st);
    }
    if (e != hipSuccess) return PIC_EDEVICE;
    S.grouped = false;
    S.counts_ready = false;
    return PIC_OK;
}

int32_t sort_box(pic_box* b)
{
    if (b->deposit_pending) return PIC_ESTATE;  // the unfused deposit reads this sort's slots
    if (side_join(b)) return PIC_EDEVICE;
    for (int s = 0; s < b->nsp; s++)
        if (sort_species(b, s, b->st)) return PIC_EDEVICE;
    b->sorted = true;
    return PIC_OK;
}

int floor_div(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// Tile y shifts of particles crossing the x faces of the shearing box in the push that uses
// dys_int = floor(Delta y_s(t^{n+1})): the new y tile is within one of (old tile + shift).
void set_migration_shift(pic_box* b, int dys_int)
{
    if (!sheared(&b->d)) {
        b->mg.cy_out = b->mg.cy_in = 0;
        return;
    }
    const int TY = b->tile[1], nty = b->tl.nt[1];
    auto wrap = [&](int v) { return ((v % nty) + nty) % nty; };
    b->mg.cy_out = wrap(floor_div(dys_int - 1, TY) + 1);
    b->mg.cy_in = wrap(floor_div(-dys_int - 2, TY) + 1);
}

int32_t zero_current(pic_box* b)
{
    for (int c = 0; c < 3; c++)
        if (zero_floats(b->J[c] - b->origin, b->comp_elems, b->st) != hipSuccess) return PIC_EDEVICE;
    return PIC_OK;
}

int32_t push_box(pic_box* b, bool fuse)
{
    if (side_join(b)) return PIC_EDEVICE;
    if (!b->sorted) return PIC_ESTATE;
    if (fuse) {
        int32_t r = zero_current(b);
        if (r) return r;
    } else {
        // workspace of the unfused deposit (old position and deposit displacement per slot)
        for (int s = 0; s < b->nsp; s++) {
            Species& S = b->sp[s];
            if (S.ws_cell) continue;
            const size_t cap = (size_t)S.cap + 1;
            int32_t r = dalloc(b, S.ws_cell, cap);
            for (int c = 0; c < 3 && !r; c++) r = dalloc(b, S.ws_off[c], cap);
            for (int c = 0; c < 3 && !r; c++) r = dalloc(b, S.ws_disp[c], cap);
            if (r) return r;
        }
    }
    StepDev P = make_step(b);
    for (int s = 0; P.count_mig && s < b->nsp; s++)
        if (set_i32(b->sp[s].sb.fallback, 0, b->st) != hipSuccess) return PIC_EDEVICE;
    if (launch_gather_push(P, b->tile, fuse ? 1 : 0, b->st) != hipSuccess) return PIC_EDEVICE;
    for (int s = 0; s < b->nsp; s++) {
        b->sp[s].cur ^= 1;
        b->sp[s].grouped = true;
        b->sp[s].counts_ready = P.count_mig != 0;
    }
    b->sorted = false;
    b->deposit_pending = !fuse;
    b->record_valid = !fuse;
    return PIC_OK;
}

int32_t deposit_box(pic_box* b)
{
    if (side_join(b)) return PIC_EDEVICE;
    if (!b->deposit_pending) return PIC_ESTATE;
    int32_t r = zero_current(b);
    if (r) return r;
    // the saved slots and tile offsets belong to the sort before the push
    StepDev P = make_step(b);
    if (launch_deposit(P, b->tile, b->st) != hipSuccess) return PIC_EDEVICE;
    b->deposit_pending = false;
    return PIC_OK;
}

float* const* field_ptrs(pic_box* b) { return b->set[b->cur_set]; }

int32_t fill_field_guards(pic_box* b, double t)
{
    return hip_fail(fill_guards(b->G, field_ptrs(b), 6, sheared(&b->d) ? 1 : 0,
                                shear_offset(b, t), b->st));
}

int32_t fold_box(pic_box* b)
{
    const double th = time_of(b, b->step) + 0.5 * b->d.dt;
    const int shear = sheared(&b->d) ? 1 : 0;
    if (fold_current(b->G, b->J, b->Jt, shear, b->d.shear_s * b->d.shear_omega0, b->d.dt,
                     shear_offset(b, th), b->st) != hipSuccess)
        return PIC_EDEVICE;
    if (shear)  // the folded current was written into the second array: it becomes the current
        for (int c = 0; c < 3; c++) std::swap(b->J[c], b->Jt[c]);
    return PIC_OK;
}

// finalize record of a tolerance-mode step whose last sweep writes set `last`: the iterate of
// an earlier converged sweep is copied there from the other iterate set when needed
KsbFin ksb_fin(const pic_box* b, int K, int last)
{
    const int sn = b->cur_set, sb2 = (sn + 2) % 3;
    KsbFin F{};
    F.G = b->G;
    F.conv = b->conv;
    F.sweeps = reinterpret_cast<int32_t*>(b->conv + 2 * kKsbMaxSweeps);
    F.err = b->err;
    F.tol = (float)b->d.maxwell_tol;
    F.K = K;
    const int other = last == sb2 ? sn : sb2;
    for (int c = 0; c < 6; c++) {
        F.src[c] = b->set[other][c];
        F.dst[c] = b->set[last][c];
    }
    return F;
}

// The combined frame's Maxwell step runs on the expanding-frame fields (l/l_c) F_c: the factors
// that convert F^n at t^n (fwd) and back at t^{n+1} (back), the curl factors l_c^2/l (dfac) and
// kz = (l_y/l_z)^2, all at the step's times
struct CombFactors {
    float fwd[3], back[3], dfac[3], kz;
};
CombFactors comb_factors(const pic_box* b)
{
    const double dt = b->d.dt, tn = time_of(b, b->step), th = tn + 0.5 * dt, t1 = tn + dt;
    double ln[3], lh[3], l1[3];
    for (int c = 0; c < 3; c++) {
        ln[c] = scale_of(b, c, tn);
        lh[c] = scale_of(b, c, th);
        l1[c] = scale_of(b, c, t1);
    }
    const double elln = ln[0] * ln[1] * ln[2], ellh = lh[0] * lh[1] * lh[2];
    const double ell1 = l1[0] * l1[1] * l1[2];
    CombFactors f{};
    for (int c = 0; c < 3; c++) {
        f.fwd[c] = (float)(elln / ln[c]);
        f.back[c] = (float)(l1[c] / ell1);
        f.dfac[c] = (float)(lh[c] * lh[c] / ellh);
    }
    f.kz = (float)((lh[1] / lh[2]) * (lh[1] / lh[2]));
    return f;
}

int32_t maxwell_box(pic_box* b)
{
    const double dt = b->d.dt;
    const double tn = time_of(b, b->step), th = tn + 0.5 * dt, t1 = tn + dt;
    hipStream_t st = b->st;
    if (sheared(&b->d)) {
        // implicit midpoint by fixed-point sweeps from F^0 = F^n (with its own guards, at
        // t^n); every later iterate has its x images at t^{n+1}.  Three field sets: F^n (free
        // once the first sweep has read it), C, and the iterates alternating with F^n's set.
        const int K = b->d.maxwell_iters > 0 ? b->d.maxwell_iters : 8;
        const int sn = b->cur_set, sc = (sn + 1) % 3, sb2 = (sn + 2) % 3;
        const double dys1 = shear_offset(b, t1);
        const double dys0 = shear_offset(b, tn);
        const bool tol = b->d.maxwell_tol > 0.0;
        // combined frame: the sweeps run on the expanding-frame fields (l/l_c) F_c, converted
        // from F^n at t^n here and back at t^{n+1} after the last sweep, with the curl factors
        // l_c^2/l and kz = (l_y/l_z)^2 at t^{n+1/2}; one-thread-per-cell sweeps only
        const bool comb = b->d.frame == PIC_FRAME_SHEAR_EXPAND;
        float back[3] = {1.f, 1.f, 1.f}, dfac[3] = {1.f, 1.f, 1.f}, kz = 1.f;
        if (comb) {
            const CombFactors f = comb_factors(b);
            for (int c = 0; c < 3; c++) {
                back[c] = f.back[c];
                dfac[c] = f.dfac[c];
            }
            kz = f.kz;
            if (scale_fields(b->G, b->set[sn], f.fwd, st) != hipSuccess ||
                fill_guards(b->G, b->set[sn], 6, 1, dys0, st) != hipSuccess)
                return PIC_EDEVICE;
        }
        const bool staged = ksb_staged(b->G) && !comb;
        if (tol && zero_floats(reinterpret_cast<float*>(b->conv), 2 * K, st) != hipSuccess)
            return PIC_EDEVICE;
        int sk = sn, so = sb2;
        // fixed count on the staged 3D grids: two sweeps per pass over memory (the same
        // iterates bit for bit), a last single sweep when the count is odd
        const bool paired = !tol && !comb && ksb_pass_fits(b->G) && K >= 2;
        for (int k = 0; k < K; k++) {
            const bool pass = paired && k + 1 < K;
            KsbDev Kd{};
            Kd.G = b->G;
            for (int c = 0; c < 6; c++) {
                Kd.Fk[c] = b->set[sk][c];
                Kd.C[c] = b->set[sc][c];
                Kd.Fo[c] = b->set[so][c];
            }
            for (int c = 0; c < 3; c++) Kd.J[c] = b->J[c];
            Kd.dt = (float)dt;
            Kd.sO = (float)(b->d.shear_s * b->d.shear_omega0);
            Kd.half_nx = 0.5f * (float)b->n[0];
            {
                const double dys = k == 0 ? dys0 : dys1, fl = std::floor(dys);
                Kd.ydys_int = (int)fl;
                Kd.ydys_w = (float)(dys - fl);
            }
            if (tol) {
                Kd.conv = b->conv;
                Kd.tol = (float)b->d.maxwell_tol;
                Kd.k = k;
            }
            Kd.expand = comb ? 1 : 0;
            for (int c = 0; c < 3; c++) Kd.dfac[c] = dfac[c];
            Kd.kz = kz;
            if (pass) {
                const double fl = std::floor(dys1);
                Kd.y1_int = (int)fl;
                Kd.y1_w = (float)(dys1 - fl);
                if (ksb_pass(Kd, k == 0, st) != hipSuccess) return PIC_EDEVICE;
                k++;
            } else if ((staged ? ksb_sweep(Kd, k == 0, st) : ksb_sweep_unstaged(Kd, k == 0, st)) != hipSuccess) {
                return PIC_EDEVICE;
            }
            if (tol && k == K - 1 && ksb_finalize(ksb_fin(b, K, so), st) != hipSuccess)
                return PIC_EDEVICE;
            // the staged 3D sweep reads its whole halo at the (shearing-)periodic images: then
            // only the last iterate's guards are filled (for the push)
            if ((!staged || k == K - 1) && fill_guards(b->G, b->set[so], 6, 1, dys1, st) != hipSuccess)
                return PIC_EDEVICE;
            sk = so;
            so = so == sb2 ? sn : sb2;
        }
        if (comb && (scale_fields(b->G, b->set[sk], back, st) != hipSuccess ||
                     fill_guards(b->G, b->set[sk], 6, 1, dys1, st) != hipSuccess))
            return PIC_EDEVICE;
        b->cur_set = sk;
        b->last_sweeps = tol ? -1 : K;
        return PIC_OK;
    }
    // Yee: B half step, E full step, B half step, with the expanding-box factors
    double ln[3], lh[3], l1[3];
    for (int k = 0; k < 3; k++) {
        ln[k] = scale_of(b, k, tn);
        lh[k] = scale_of(b, k, th);
        l1[k] = scale_of(b, k, t1);
    }
    const double elln = ln[0] * ln[1] * ln[2], ellh = lh[0] * lh[1] * lh[2], ell1 = l1[0] * l1[1] * l1[2];
    MaxwellDev M{};
    M.G = b->G;
    for (int c = 0; c < 3; c++) {
        M.E[c] = b->E(c);
        M.B[c] = b->B(c);
        M.J[c] = b->J[c];
    }
    M.dt = (float)dt;
    float* Bp[3] = {b->B(0), b->B(1), b->B(2)};
    float* Ep[3] = {b->E(0), b->E(1), b->E(2)};
    // B'^{n+1/2} = B'^n - dt/2 curl(L^n E^n), B^{n+1/2} = (l/ell)^{n+1/2} B'
    for (int c = 0; c < 3; c++) {
        M.fin[c] = (float)(elln / ln[c]);
        M.fout[c] = (float)(lh[c] / ellh);
        M.gf[c] = (float)ln[c];
    }
    if (yee_b(M, st) != hipSuccess) return PIC_EDEVICE;
    if (fill_guards(b->G, Bp, 3, 0, 0.0, st) != hipSuccess) return PIC_EDEVICE;
    // E'^{n+1} = E'^n + dt curl(L^{n+1/2} B^{n+1/2}) - 4 pi dt (l J'), E^{n+1} = (l/ell)^{n+1} E'
    for (int c = 0; c < 3; c++) {
        M.fin[c] = (float)(elln / ln[c]);
        M.fout[c] = (float)(l1[c] / ell1);
        M.gf[c] = (float)lh[c];
    }
    if (yee_e(M, st) != hipSuccess) return PIC_EDEVICE;
    if (fill_guards(b->G, Ep, 3, 0, 0.0, st) != hipSuccess) return PIC_EDEVICE;
    // B'^{n+1} = B'^{n+1/2} - dt/2 curl(L^{n+1} E^{n+1}), B^{n+1} = (l/ell)^{n+1} B'
    for (int c = 0; c < 3; c++) {
        M.fin[c] = (float)(ellh / lh[c]);
        M.fout[c] = (float)(l1[c] / ell1);
        M.gf[c] = (float)l1[c];
    }
    if (yee_b(M, st) != hipSuccess) return PIC_EDEVICE;
    if (fill_guards(b->G, Bp, 3, 0, 0.0, st) != hipSuccess) return PIC_EDEVICE;
    return PIC_OK;
}

// ---------------------------------------------------------------- batched step
// pic_step over many boxes: every stage of the step (sort, current zeroing, push, fold, Maxwell,
// guard fill) is one launch per kernel for all boxes, driven by tables of per-box arguments.
// The tables of a whole step are staged on the host, copied to the device in one transfer and
// then launched stage by stage on the shared stream.
struct BatchPlan {
    hipStream_t st = nullptr;
    std::vector<char> buf;
    std::vector<std::function<hipError_t(const char*)>> launches;
    std::vector<uint64_t> sig;  // launch sequence: kind, table offsets, units, blocks, shape
    void note(uint64_t kind, size_t to, size_t po, int nu, int total, uint64_t extra)
    {
        sig.insert(sig.end(), {kind, (uint64_t)to, (uint64_t)po, (uint64_t)nu, (uint64_t)total, extra});
    }

    size_t put(const void* p, size_t bytes)
    {
        const size_t off = (buf.size() + 255) & ~(size_t)255;
        buf.resize(off + bytes);
        std::memcpy(buf.data() + off, p, bytes);
        return off;
    }
    // one table + prefix; returns false if the stage has no blocks
    template <class Args>
    bool stage(const std::vector<Args>& a, const std::vector<uint32_t>& blocks, size_t& to,
               size_t& po, int& total)
    {
        if (a.empty()) return false;
        std::vector<uint32_t> prefix(a.size() + 1, 0);
        for (size_t i = 0; i < a.size(); i++) prefix[i + 1] = prefix[i] + blocks[i];
        if (prefix.back() == 0) return false;
        to = put(a.data(), sizeof(Args) * a.size());
        po = put(prefix.data(), sizeof(uint32_t) * prefix.size());
        total = (int)prefix.back();
        return true;
    }
    template <class Args>
    void grid(GridBatchKind k, const std::vector<Args>& a, const std::vector<uint32_t>& blocks, int ydim)
    {
        size_t to, po;
        int total;
        if (!stage(a, blocks, to, po, total)) return;
        const int nu = (int)a.size();
        note(100 + (uint64_t)k, to, po, nu, total, (uint64_t)ydim);
        hipStream_t s = st;
        launches.push_back([=](const char* d) {
            return grid_batch(k, d + to, UnitMap{reinterpret_cast<const uint32_t*>(d + po), nu}, total,
                              ydim, s);
        });
    }
    template <class Args>
    void sort(SortBatchKind k, const std::vector<Args>& a, const std::vector<uint32_t>& blocks)
    {
        size_t to, po;
        int total;
        if (!stage(a, blocks, to, po, total)) return;
        const int nu = (int)a.size();
        note(200 + (uint64_t)k, to, po, nu, total, 0);
        hipStream_t s = st;
        launches.push_back([=](const char* d) {
            return sort_batch(k, d + to, UnitMap{reinterpret_cast<const uint32_t*>(d + po), nu}, total, s);
        });
    }
    void push(const std::vector<StepDev>& a, const std::vector<uint32_t>& blocks, int dim,
              const int tile[3], int frame)
    {
        size_t to, po;
        int total;
        if (!stage(a, blocks, to, po, total)) return;
        const int nu = (int)a.size();
        const int t[3] = {tile[0], tile[1], tile[2]};
        note(300, to, po, nu, total,
             (uint64_t)dim | (uint64_t)tile[0] << 8 | (uint64_t)tile[1] << 16 | (uint64_t)tile[2] << 24 |
                 (uint64_t)frame << 32);
        hipStream_t s = st;
        launches.push_back([=](const char* d) {
            return launch_gather_push_batch(reinterpret_cast<const StepDev*>(d + to),
                                            UnitMap{reinterpret_cast<const uint32_t*>(d + po), nu},
                                            total, dim, t, frame, s);
        });
    }
};

// guard fill of ncomp arrays as batched units (one per slab kind)
void plan_fill(std::vector<FillArgs>& a, std::vector<uint32_t>& blk, const GridDev& G,
               float* const* comps, int ncomp, int shear, double dys)
{
    Comp6 A{};
    for (int c = 0; c < ncomp; c++) A.p[c] = comps[c];
    const double fl = std::floor(dys);
    const int di = (int)fl;
    const float w = (float)(dys - fl);
    const int NYg = G.n[1] + 2 * G.g[1], NZg = G.n[2] + 2 * G.g[2];
    a.push_back(FillArgs{G, A, 0, shear, di, w});
    blk.push_back(grid_blocks((int64_t)2 * G.g[0] * NYg * NZg));
    a.push_back(FillArgs{G, A, 1, shear, di, w});
    blk.push_back(grid_blocks((int64_t)G.n[0] * 2 * G.g[1] * NZg));
    if (G.g[2] > 0) {
        a.push_back(FillArgs{G, A, 2, shear, di, w});
        blk.push_back(grid_blocks((int64_t)G.n[0] * G.n[1] * 2 * G.g[2]));
    }
}

// The host-side state a batched step advances, per box: saved before planning so that a step
// whose tables do not fit caller-owned staging (or a dry run that only measures the tables)
// leaves every box as it was.
struct BoxState {
    bool sorted, deposit_pending, record_valid;
    int64_t step, n_migrations;
    int cur_set, last_sweeps;
    float* J[3];
    float* Jt[3];
    MigGeo mg;  // the y shifts of the last push's face crossings, read by the next sort
    struct Sp {
        int cur, toff_cur, which, n_upper;
        bool grouped, counts_ready;
    } sp[kMaxSpecies];
};
BoxState save_state(const pic_box* b)
{
    BoxState v{};
    v.sorted = b->sorted;
    v.deposit_pending = b->deposit_pending;
    v.record_valid = b->record_valid;
    v.step = b->step;
    v.n_migrations = b->n_migrations;
    v.cur_set = b->cur_set;
    v.last_sweeps = b->last_sweeps;
    v.mg = b->mg;
    for (int c = 0; c < 3; c++) {
        v.J[c] = b->J[c];
        v.Jt[c] = b->Jt[c];
    }
    for (int s = 0; s < b->nsp; s++) {
        const Species& S = b->sp[s];
        v.sp[s] = BoxState::Sp{S.cur, S.toff_cur, S.which, S.n_upper, S.grouped, S.counts_ready};
    }
    return v;
}
void restore_state(pic_box* b, const BoxState& v)
{
    b->sorted = v.sorted;
    b->deposit_pending = v.deposit_pending;
    b->record_valid = v.record_valid;
    b->step = v.step;
    b->n_migrations = v.n_migrations;
    b->cur_set = v.cur_set;
    b->last_sweeps = v.last_sweeps;
    b->mg = v.mg;
    for (int c = 0; c < 3; c++) {
        b->J[c] = v.J[c];
        b->Jt[c] = v.Jt[c];
    }
    for (int s = 0; s < b->nsp; s++) {
        Species& S = b->sp[s];
        S.cur = v.sp[s].cur;
        S.toff_cur = v.sp[s].toff_cur;
        S.which = v.sp[s].which;
        S.n_upper = v.sp[s].n_upper;
        S.grouped = v.sp[s].grouped;
        S.counts_ready = v.sp[s].counts_ready;
    }
}

// One batched step of the boxes, its tables staged in sg.  dry: only measure the tables
// (*table_bytes), queue nothing and leave the boxes as they were.
int32_t step_batched(pic_box* const* boxes, int nb, bool graph, Stager& sg_all, bool dry,
                     size_t* table_bytes)
{
    hipStream_t st = boxes[0]->st;
    for (int i = 0; i < nb; i++) {
        pic_box* b = boxes[i];
        if (b->st != st || b->deposit_pending) return b->st != st ? PIC_EINVAL : PIC_ESTATE;
        if (!batch_tile_supported(b->dim, b->tile)) return PIC_EINVAL;
        for (int j = 0; j < i; j++)
            if (boxes[j] == b) return PIC_EINVAL;
    }
    BatchPlan plan;
    plan.st = st;
    std::vector<BoxState> saved(nb);
    for (int i = 0; i < nb; i++) saved[i] = save_state(boxes[i]);
    auto undo = [&](int32_t r) {
        for (int i = 0; i < nb; i++) restore_state(boxes[i], saved[i]);
        return r;
    };

    // ---- a1: tile sort (migration sort in the batch; radix per box where it does not apply)
    {
        std::vector<ZeroArgs> zf;
        std::vector<uint32_t> zfb;
        std::vector<MigCountArgs> mc;
        std::vector<MigOffArgs> mo;
        std::vector<ScanArgs> sc;
        std::vector<MigScatterArgs> ms;
        std::vector<uint32_t> mcb, mob, scb, msb;
        std::vector<int> radix_boxes;
        for (int i = 0; i < nb; i++) {
            pic_box* b = boxes[i];
            bool all_grouped = b->mig_ok;
            for (int s = 0; s < b->nsp; s++) all_grouped = all_grouped && b->sp[s].grouped;
            if (!all_grouped) {
                radix_boxes.push_back(i);
                continue;
            }
            const int nt = b->tl.n_tiles;
            for (int s = 0; s < b->nsp; s++) {
                Species& S = b->sp[s];
                const int nxt = S.toff_cur ^ 1;
                const Gate g{S.sb.fallback, 0};
                S.which = sort_result_buffer(b->tl);
                if (!S.counts_ready) {  // else the push wrote the counts and the flag
                    zf.push_back(ZeroArgs{reinterpret_cast<uint32_t*>(S.sb.fallback), 1});
                    zfb.push_back(1);
                    mc.push_back(MigCountArgs{S.cell[S.cur], S.toff[S.toff_cur], b->cc, b->mg,
                                              S.sb.mcnt, S.sb.fallback, b->err});
                    mcb.push_back((uint32_t)nt);
                }
                S.counts_ready = false;
                mo.push_back(MigOffArgs{S.sb.mcnt, b->mg, S.sb.mpre, S.sb.tot, S.sb.dcnt, g});
                mob.push_back((uint32_t)((nt + kBlock / 64 - 1) / (kBlock / 64)));
                sc.push_back(ScanArgs{S.sb.tot, S.sb.start, nt + 1, g});
                scb.push_back(1);
                sc.push_back(ScanArgs{S.sb.dcnt, S.sb.dpre, nt + 1, g});
                scb.push_back(1);
                ms.push_back(MigScatterArgs{S.cell[S.cur], S.toff[S.toff_cur], S.n_upper, b->cc, b->mg,
                                            S.sb.mpre, S.sb.start, S.sb.dpre, S.sb.vals[S.which],
                                            S.toff[nxt], S.n_live, g});
                msb.push_back((uint32_t)(nt + 1));
                S.toff_cur = nxt;
                S.grouped = false;
                b->n_migrations++;
            }
            b->sorted = true;
        }
        // boxes the migration sort does not apply to are sorted now, on their own launches,
        // ahead of the batch on the shared stream (a dry run only marks them sorted)
        for (int i : radix_boxes) {
            if (dry) {
                boxes[i]->sorted = true;
                for (int s = 0; s < boxes[i]->nsp; s++)
                    boxes[i]->sp[s].grouped = boxes[i]->sp[s].counts_ready = false;
                continue;
            }
            if (sort_box(boxes[i])) return undo(PIC_EDEVICE);
        }
        plan.grid(kBatchZero, zf, zfb, 1);
        plan.sort(kBatchMigCount, mc, mcb);
        plan.sort(kBatchMigOffsets, mo, mob);
        plan.sort(kBatchScan, sc, scb);
        plan.sort(kBatchMigScatter, ms, msb);
    }

    // ---- current zeroing and the fused push (a2-a6, a8)
    {
        std::vector<ZeroArgs> z;
        std::vector<uint32_t> zb;
        std::map<std::tuple<int, int, int, int, int>, std::pair<std::vector<StepDev>, std::vector<uint32_t>>> groups;
        for (int i = 0; i < nb; i++) {
            pic_box* b = boxes[i];
            for (int c = 0; c < 3; c++) {
                z.push_back(ZeroArgs{reinterpret_cast<uint32_t*>(b->J[c] - b->origin), b->comp_elems});
                zb.push_back(grid_blocks(b->comp_elems));
            }
            auto& gr = groups[std::make_tuple(b->dim, b->tile[0], b->tile[1], b->tile[2], b->d.frame)];
            StepDev P = make_step(b);
            P.mig_latch = 1;  // no radix fallback behind a batched sort
            gr.first.push_back(P);
            gr.second.push_back((uint32_t)b->tl.n_tiles);
            for (int s = 0; s < b->nsp; s++) {
                if (P.count_mig) {  // cleared after this step's sort read it, set by the push
                    z.push_back(ZeroArgs{reinterpret_cast<uint32_t*>(b->sp[s].sb.fallback), 1});
                    zb.push_back(1);
                }
                b->sp[s].cur ^= 1;
                b->sp[s].grouped = true;
                b->sp[s].counts_ready = P.count_mig != 0;
            }
            b->sorted = false;
            b->record_valid = false;
        }
        plan.grid(kBatchZero, z, zb, 1);
        for (auto& kv : groups) {
            const int tile[3] = {std::get<1>(kv.first), std::get<2>(kv.first), std::get<3>(kv.first)};
            plan.push(kv.second.first, kv.second.second, std::get<0>(kv.first), tile, std::get<4>(kv.first));
        }
    }

    // ---- a7: current fold (z, y periodic; J' transport and shearing-periodic x, or periodic x)
    {
        std::vector<FoldPArgs> fz, fy;
        std::vector<ShearFoldArgs> adv;
        std::vector<FoldXArgs> fx;
        std::vector<uint32_t> fzb, fyb, advb, fxb;
        for (int i = 0; i < nb; i++) {
            pic_box* b = boxes[i];
            const GridDev& G = b->G;
            const Comp3 Jc{{b->J[0], b->J[1], b->J[2]}};
            const int NXg = G.n[0] + 2 * G.g[0], NYg = G.n[1] + 2 * G.g[1];
            if (G.g[2] > 0) {
                const int nl = G.n[2] < 2 * G.g[2] ? G.n[2] : 2 * G.g[2];
                fz.push_back(FoldPArgs{G, Jc, 2});
                fzb.push_back(grid_blocks((int64_t)NXg * NYg * nl));
            }
            const int nly = G.n[1] < 2 * G.g[1] ? G.n[1] : 2 * G.g[1];
            fy.push_back(FoldPArgs{G, Jc, 1});
            fyb.push_back(grid_blocks((int64_t)NXg * nly * G.n[2]));
            const double th = time_of(b, b->step) + 0.5 * b->d.dt;
            if (sheared(&b->d)) {
                // transport + x fold from J into the second array, which then becomes the
                // current (the later stages of this step are planned with the swapped arrays)
                const double dh = shear_offset(b, th), fl = std::floor(dh);
                const Comp3 Tc{{b->Jt[0], b->Jt[1], b->Jt[2]}};
                adv.push_back(ShearFoldArgs{G, Jc, Tc, (float)(b->d.shear_s * b->d.shear_omega0 * b->d.dt / 2.0),
                                            0.5f * G.n[0], (int)fl, (float)(dh - fl)});
                advb.push_back(grid_blocks((int64_t)G.n[0] * G.n[1] * G.n[2]));
                for (int c = 0; c < 3; c++) std::swap(b->J[c], b->Jt[c]);
            } else {
                const int nlx = G.n[0] < 2 * G.g[0] ? G.n[0] : 2 * G.g[0];
                fx.push_back(FoldXArgs{G, Jc, Jc, 0, 0, 0, 0.f});
                fxb.push_back(grid_blocks((int64_t)nlx * G.n[1] * G.n[2]));
            }
        }
        plan.grid(kBatchFoldP, fz, fzb, 3);
        plan.grid(kBatchFoldP, fy, fyb, 3);
        plan.grid(kBatchShearFold, adv, advb, 3);
        plan.grid(kBatchFoldX, fx, fxb, 3);
    }

    // ---- a9: Maxwell (Yee with the expanding-box factors; shearing-box fixed-point sweeps)
    {
        std::vector<MaxwellDev> yb1, ye, yb2;
        std::vector<uint32_t> yb1b, yeb, yb2b;
        std::vector<FillArgs> fb1, fe, fb2, fend;
        std::vector<uint32_t> fb1b, feb, fb2b, fendb;
        int kmax = 0;
        for (int i = 0; i < nb; i++) {
            pic_box* b = boxes[i];
            if (sheared(&b->d)) {
                kmax = std::max(kmax, b->d.maxwell_iters > 0 ? b->d.maxwell_iters : 8);
                continue;
            }
            const double dt = b->d.dt, tn = time_of(b, b->step), th = tn + 0.5 * dt, t1 = tn + dt;
            double ln[3], lh[3], l1[3];
            for (int k = 0; k < 3; k++) {
                ln[k] = scale_of(b, k, tn);
                lh[k] = scale_of(b, k, th);
                l1[k] = scale_of(b, k, t1);
            }
            const double elln = ln[0] * ln[1] * ln[2], ellh = lh[0] * lh[1] * lh[2],
                         ell1 = l1[0] * l1[1] * l1[2];
            MaxwellDev M{};
            M.G = b->G;
            for (int c = 0; c < 3; c++) {
                M.E[c] = b->E(c);
                M.B[c] = b->B(c);
                M.J[c] = b->J[c];
            }
            M.dt = (float)dt;
            const uint32_t nbk = grid_blocks((int64_t)b->n[0] * b->n[1] * b->n[2]);
            float* Bp[3] = {b->B(0), b->B(1), b->B(2)};
            float* Ep[3] = {b->E(0), b->E(1), b->E(2)};
            for (int c = 0; c < 3; c++) {
                M.fin[c] = (float)(elln / ln[c]);
                M.fout[c] = (float)(lh[c] / ellh);
                M.gf[c] = (float)ln[c];
            }
            yb1.push_back(M);
            yb1b.push_back(nbk);
            plan_fill(fb1, fb1b, b->G, Bp, 3, 0, 0.0);
            for (int c = 0; c < 3; c++) {
                M.fin[c] = (float)(elln / ln[c]);
                M.fout[c] = (float)(l1[c] / ell1);
                M.gf[c] = (float)lh[c];
            }
            ye.push_back(M);
            yeb.push_back(nbk);
            plan_fill(fe, feb, b->G, Ep, 3, 0, 0.0);
            for (int c = 0; c < 3; c++) {
                M.fin[c] = (float)(ellh / lh[c]);
                M.fout[c] = (float)(l1[c] / ell1);
                M.gf[c] = (float)l1[c];
            }
            yb2.push_back(M);
            yb2b.push_back(nbk);
            plan_fill(fb2, fb2b, b->G, Bp, 3, 0, 0.0);
        }
        plan.grid(kBatchYeeB, yb1, yb1b, 1);
        plan.grid(kBatchFill, fb1, fb1b, 3);
        plan.grid(kBatchYeeE, ye, yeb, 1);
        plan.grid(kBatchFill, fe, feb, 3);
        plan.grid(kBatchYeeB, yb2, yb2b, 1);
        plan.grid(kBatchFill, fb2, fb2b, 3);
        // shearing boxes: sweep k of every box with at least k+1 sweeps in one launch
        struct Rot {
            int sn, sc, sb2, sk, so;
        };
        std::vector<Rot> rot(nb);
        for (int i = 0; i < nb; i++) {
            pic_box* b = boxes[i];
            const int sn = b->cur_set;
            rot[i] = Rot{sn, (sn + 1) % 3, (sn + 2) % 3, sn, (sn + 2) % 3};
        }
        // combined-frame boxes: F^n to the expanding-frame fields at t^n, guards at t^n
        std::vector<CombFactors> cf(nb);
        {
            std::vector<ScaleArgs> sa;
            std::vector<uint32_t> sab;
            std::vector<FillArgs> sf;
            std::vector<uint32_t> sfb;
            for (int i = 0; i < nb; i++) {
                pic_box* b = boxes[i];
                if (b->d.frame != PIC_FRAME_SHEAR_EXPAND) continue;
                cf[i] = comb_factors(b);
                ScaleArgs a{};
                a.G = b->G;
                for (int c = 0; c < 6; c++) a.F[c] = b->set[rot[i].sn][c];
                for (int c = 0; c < 3; c++) a.f[c] = cf[i].fwd[c];
                sa.push_back(a);
                sab.push_back(grid_blocks((int64_t)b->n[0] * b->n[1] * b->n[2]));
                plan_fill(sf, sfb, b->G, b->set[rot[i].sn], 6, 1, shear_offset(b, time_of(b, b->step)));
            }
            plan.grid(kBatchScale, sa, sab, 1);
            plan.grid(kBatchFill, sf, sfb, 6);
        }
        // tolerance-mode boxes: clear their convergence records first
        {
            std::vector<ZeroArgs> cz;
            std::vector<uint32_t> czb;
            for (int i = 0; i < nb; i++) {
                pic_box* b = boxes[i];
                if (!sheared(&b->d) || !(b->d.maxwell_tol > 0.0)) continue;
                const int K = b->d.maxwell_iters > 0 ? b->d.maxwell_iters : 8;
                cz.push_back(ZeroArgs{b->conv, (int64_t)2 * K});
                czb.push_back(grid_blocks(2 * K));
            }
            plan.grid(kBatchZero, cz, czb, 1);
        }
        for (int k = 0; k < kmax; k++) {
            std::vector<KsbDev> ks;
            std::vector<uint32_t> ksb;
            std::vector<FillArgs> kf;
            std::vector<uint32_t> kfb;
            std::vector<KsbFin> kz;
            std::vector<uint32_t> kzb;
            for (int i = 0; i < nb; i++) {
                pic_box* b = boxes[i];
                if (!sheared(&b->d)) continue;
                const int K = b->d.maxwell_iters > 0 ? b->d.maxwell_iters : 8;
                if (k >= K) continue;
                const bool tol = b->d.maxwell_tol > 0.0;
                Rot& r = rot[i];
                KsbDev Kd{};
                Kd.G = b->G;
                for (int c = 0; c < 6; c++) {
                    Kd.Fk[c] = b->set[r.sk][c];
                    Kd.C[c] = b->set[r.sc][c];
                    Kd.Fo[c] = b->set[r.so][c];
                }
                for (int c = 0; c < 3; c++) Kd.J[c] = b->J[c];
                Kd.dt = (float)b->d.dt;
                Kd.sO = (float)(b->d.shear_s * b->d.shear_omega0);
                Kd.half_nx = 0.5f * (float)b->n[0];
                if (tol) {
                    Kd.conv = b->conv;
                    Kd.tol = (float)b->d.maxwell_tol;
                    Kd.k = k;
                }
                if (b->d.frame == PIC_FRAME_SHEAR_EXPAND) {
                    Kd.expand = 1;
                    for (int c = 0; c < 3; c++) Kd.dfac[c] = cf[i].dfac[c];
                    Kd.kz = cf[i].kz;
                } else {
                    for (int c = 0; c < 3; c++) Kd.dfac[c] = 1.f;
                    Kd.kz = 1.f;
                }
                ks.push_back(Kd);
                ksb.push_back(grid_blocks((int64_t)b->n[0] * b->n[1] * b->n[2]));
                if (tol && k == K - 1) {
                    kz.push_back(ksb_fin(b, K, r.so));
                    kzb.push_back(kKsbFinBlocks);
                }
                const double t1 = time_of(b, b->step) + b->d.dt;
                plan_fill(kf, kfb, b->G, b->set[r.so], 6, 1, shear_offset(b, t1));
                r.sk = r.so;
                r.so = r.so == r.sb2 ? r.sn : r.sb2;
                if (k == K - 1) {
                    b->cur_set = r.sk;
                    b->last_sweeps = tol ? -1 : K;
                }
            }
            plan.grid(k == 0 ? kBatchKsbFirst : kBatchKsbNext, ks, ksb, 1);
            plan.grid(kBatchKsbFinal, kz, kzb, 1);
            plan.grid(kBatchFill, kf, kfb, 6);
        }
        // combined-frame boxes: the last iterate back to the frame's fields at t^{n+1}
        {
            std::vector<ScaleArgs> sa;
            std::vector<uint32_t> sab;
            for (int i = 0; i < nb; i++) {
                pic_box* b = boxes[i];
                if (b->d.frame != PIC_FRAME_SHEAR_EXPAND) continue;
                ScaleArgs a{};
                a.G = b->G;
                for (int c = 0; c < 6; c++) a.F[c] = b->set[b->cur_set][c];
                for (int c = 0; c < 3; c++) a.f[c] = cf[i].back[c];
                sa.push_back(a);
                sab.push_back(grid_blocks((int64_t)b->n[0] * b->n[1] * b->n[2]));
                plan_fill(fend, fendb, b->G, b->set[b->cur_set], 6, 1,
                          shear_offset(b, time_of(b, b->step) + b->d.dt));
            }
            plan.grid(kBatchScale, sa, sab, 1);
        }
        // time advance; guard cells of the non-shear fields at t^{n+1}
        for (int i = 0; i < nb; i++) {
            pic_box* b = boxes[i];
            b->step += 1;
            if (!sheared(&b->d)) plan_fill(fend, fendb, b->G, field_ptrs(b), 6, 0, 0.0);
        }
        plan.grid(kBatchFill, fend, fendb, 6);
    }

    // ---- stage the tables, one transfer, then the launches in order
    const size_t bytes = plan.buf.size();
    if (dry) {
        *table_bytes = bytes;
        return undo(PIC_OK);
    }
    const int sidx = sg_all.cur;
    auto& sg = sg_all.buf[sidx];
    if (bytes > sg.cap) {
        if (sg_all.caller) return undo(PIC_ENOMEM);  // caller-owned staging is never grown
        if (sg.copied && hipEventSynchronize(sg.copied) != hipSuccess) return PIC_EDEVICE;
        if (hipStreamSynchronize(st) != hipSuccess) return PIC_EDEVICE;  // the old tables may be in use
        lib_host_free(sg.host, sg.cap);
        lib_free(sg.dev, sg.cap);
        sg.host = sg.dev = nullptr;
        for (auto& g : sg_all.graphs) hipGraphExecDestroy(g.exec);  // they read the old buffer
        sg_all.graphs.clear();
        sg.cap = 0;
        const size_t cap = std::max(bytes * 2, (size_t)1 << 20);
        if (lib_host_malloc(&sg.host, cap) != hipSuccess) return PIC_ENOMEM;
        if (lib_malloc(&sg.dev, cap) != hipSuccess) {
            lib_host_free(sg.host, cap);
            sg.host = nullptr;
            return PIC_ENOMEM;
        }
        sg.cap = cap;
    } else if (sg.copied && hipEventSynchronize(sg.copied) != hipSuccess) {
        return PIC_EDEVICE;
    }
    if (!sg.copied && hipEventCreateWithFlags(&sg.copied, hipEventDisableTiming) != hipSuccess)
        return PIC_EDEVICE;
    sg_all.cur ^= 1;
    if (bytes) std::memcpy(sg.host, plan.buf.data(), bytes);
    const char* dev = static_cast<const char*>(sg.dev);
    auto enqueue = [&]() -> int32_t {
        if (bytes && hipMemcpyAsync(sg.dev, sg.host, bytes, hipMemcpyHostToDevice, st) != hipSuccess)
            return PIC_EDEVICE;
        for (auto& f : plan.launches)
            if (f(dev) != hipSuccess) return PIC_EDEVICE;
        return PIC_OK;
    };
    if (!graph || !bytes) {
        if (enqueue()) return PIC_EDEVICE;
        if (bytes && hipEventRecord(sg.copied, st) != hipSuccess) return PIC_EDEVICE;
        return PIC_OK;
    }
    // graph mode: the step's transfer and launches form one graph, captured the first time this
    // box set and launch sequence meet this staging buffer and replayed afterwards (the memcpy
    // node reads the tables the host has just written to the pinned buffer)
    std::vector<uint64_t> key;
    key.reserve(plan.sig.size() + nb + 4);
    key.push_back((uint64_t)sidx);
    key.push_back((uint64_t)(uintptr_t)sg.dev);
    key.push_back((uint64_t)bytes);
    for (int i = 0; i < nb; i++) key.push_back(boxes[i]->uid);
    key.insert(key.end(), plan.sig.begin(), plan.sig.end());
    auto& cache = sg_all.graphs;
    size_t hit = cache.size();
    for (size_t i = 0; i < cache.size(); i++)
        if (cache[i].key == key) {
            hit = i;
            break;
        }
    if (hit == cache.size()) {
        if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) return PIC_EDEVICE;
        const int32_t er = enqueue();
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(st, &g);
        if (er || ec != hipSuccess || !g) {
            if (g) hipGraphDestroy(g);
            return PIC_EDEVICE;
        }
        hipGraphExec_t ex = nullptr;
        const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        hipGraphDestroy(g);
        if (ei != hipSuccess) return PIC_EDEVICE;
        constexpr size_t kMaxGraphs = 8;
        if (cache.size() >= kMaxGraphs) {
            hipGraphExecDestroy(cache.back().exec);
            cache.pop_back();
        }
        cache.insert(cache.begin(), Stager::StepGraph{std::move(key), ex});
        hit = 0;
    } else if (hit != 0) {
        std::rotate(cache.begin(), cache.begin() + hit, cache.begin() + hit + 1);
        hit = 0;
    }
    if (hipGraphLaunch(cache[hit].exec, st) != hipSuccess) return PIC_EDEVICE;
    if (hipEventRecord(sg.copied, st) != hipSuccess) return PIC_EDEVICE;
    return PIC_OK;
}

// Validate the descriptor and set a new box's geometry (no device work).  pitch[2]: element
// strides of the guarded field arrays along y and z, or 0 for the smallest valid ones.
int32_t init_box(const pic_box_desc* d, const int32_t pitch[2], pic_box*& out)
{
    out = nullptr;
    if (!d) return PIC_EINVAL;
    if (d->dim != 2 && d->dim != 3) return PIC_EINVAL;
    int n[3] = {d->n[0], d->n[1], d->dim == 3 ? d->n[2] : 1};
    if (d->dim == 2 && d->n[2] != 1 && d->n[2] != 0) return PIC_EINVAL;
    for (int k = 0; k < d->dim; k++)
        if (n[k] < 4) return PIC_EINVAL;
    if (!(d->dt > 0) || d->dt * std::sqrt((double)d->dim) >= 1.0) return PIC_EINVAL;
    if (d->frame < 0 || d->frame > 4) return PIC_EINVAL;
    // the combined frame scales x and y together (axis masks 0, z, xy, xyz)
    if (d->frame == PIC_FRAME_SHEAR_EXPAND && ((d->expand_axis_mask & 3) == 1 || (d->expand_axis_mask & 3) == 2))
        return PIC_EINVAL;
    if (d->n_species < 1 || d->n_species > 2) return PIC_EINVAL;
    if (d->maxwell_iters < 0 || d->maxwell_iters > kKsbMaxSweeps || !(d->maxwell_tol >= 0.0) ||
        !(d->maxwell_tol < 1.0))
        return PIC_EINVAL;
    if (escapes(d)) {
        if (d->leaky_mode == PIC_LEAKY_DISPLACEMENT && !(d->leaky_l_esc > 0 && d->leaky_theta_inj > 0))
            return PIC_EINVAL;
        if (d->leaky_mode == PIC_LEAKY_PROBABILISTIC && !(d->leaky_t_esc > 0)) return PIC_EINVAL;
        if (d->leaky_mode != 0 && d->leaky_mode != 1) return PIC_EINVAL;
    }
    int tile[3];
    for (int k = 0; k < 3; k++) tile[k] = d->tile[k];
    if (tile[0] == 0) {
        tile[0] = tile[1] = d->dim == 3 ? 8 : 16;
        tile[2] = d->dim == 3 ? 8 : 1;
    }
    if (d->dim == 2) tile[2] = 1;
    if (!tile_shape_supported(d->dim, tile)) return PIC_EINVAL;
    int bits[3];
    for (int k = 0; k < 3; k++) bits[k] = ceil_log2(n[k]);
    if (bits[0] + bits[1] + bits[2] > 31) return PIC_EINVAL;
    for (int s = 0; s < d->n_species; s++)
        if (d->capacity[s] < 0 || d->capacity[s] >= (1ll << 30)) return PIC_EINVAL;  // 32-bit byte offsets
    // field rows of kRowAlign floats: interior x = 0 starts a 128-byte line in every row (the x
    // guards sit in the padding before and after the interior)
    const int g = kGuard, gz = d->dim == 3 ? kGuard : 0;
    const int NYg = n[1] + 2 * g, NZg = n[2] + 2 * gz;
    const int64_t sy_min = (int64_t)(kRowAlign + n[0] + g + kRowAlign - 1) / kRowAlign * kRowAlign;
    int64_t sy = sy_min, sz = sy_min * NYg;
    if (pitch && (pitch[0] || pitch[1])) {
        sy = pitch[0];
        sz = pitch[1];
        if (sy < sy_min || sy % kRowAlign || sz < sy * NYg || sz % kRowAlign) return PIC_EINVAL;
    }
    if (sz * NZg >= (1ll << 31)) return PIC_EINVAL;

    pic_box* b = new (std::nothrow) pic_box();
    if (!b) return PIC_ENOMEM;
    static std::atomic<uint64_t> next_uid{0};
    b->uid = ++next_uid;
    b->d = *d;
    b->st = static_cast<hipStream_t>(d->stream);
    b->dim = d->dim;
    for (int k = 0; k < 3; k++) b->n[k] = n[k];
    b->cc.b0 = bits[0];
    b->cc.b1 = bits[1];
    b->cc.m0 = (1u << bits[0]) - 1u;
    b->cc.m1 = (1u << bits[1]) - 1u;
    set_tiling(b, tile);
    GridDev& G = b->G;
    G.dim = b->dim;
    G.div0 = FastDiv::make((uint32_t)n[0]);
    G.div1 = FastDiv::make((uint32_t)n[1]);
    for (int k = 0; k < 3; k++) {
        G.n[k] = n[k];
        G.g[k] = (k < b->dim) ? kGuard : 0;
    }
    G.divyg = FastDiv::make((uint32_t)NYg);
    G.sy = (int)sy;
    G.sz = (int)sz;
    b->comp_elems = sz * NZg;
    b->origin = (int64_t)kRowAlign + sy * G.g[1] + sz * G.g[2];
    b->nsp = d->n_species;
    b->track_ids = (d->flags & PIC_BOX_TRACK_IDS) || escapes(d);
    b->nsets = sheared(d) ? 3 : 1;
    out = b;
    return PIC_OK;
}

bool unfused_reserved(const pic_box* b) { return (b->d.flags & PIC_BOX_UNFUSED) != 0; }

// The box's buffers.  Fields, currents and particle arrays come from the caller's pic_box_mem
// when there is one, everything else from the workspace (library allocation or caller block).
// Measuring pass (alloc_pass 1): only the workspace is counted.
int32_t alloc_all(pic_box* b, const pic_box_mem* m)
{
    const pic_box_desc* d = &b->d;
    const int tiles_ws = max_tiles(b->dim, b->n);  // any supported tiling fits the workspace
    int32_t r = PIC_OK;
    const bool measuring = b->alloc_pass == 1;
    // a buffer the caller may own: taken from m (checked: non-null, 256-byte aligned) or carved
    auto caller_buf = [&](auto*& p, auto* given, size_t count) -> int32_t {
        if (m) {
            if (measuring) return PIC_OK;
            if (!given || (reinterpret_cast<uintptr_t>(given) & 255)) return PIC_EINVAL;
            p = given;
            return PIC_OK;
        }
        return dalloc(b, p, count);
    };
    auto field = [&](float*& p, float* given) -> int32_t {
        float* q = nullptr;
        int32_t rr = caller_buf(q, given, (size_t)b->comp_elems);
        if (rr || measuring) return rr;
        if (hipMemsetAsync(q, 0, sizeof(float) * b->comp_elems, b->st) != hipSuccess) return PIC_EDEVICE;
        p = q + b->origin;
        return PIC_OK;
    };
    for (int s = 0; s < b->nsets && !r; s++)
        for (int c = 0; c < 6 && !r; c++) r = field(b->set[s][c], m ? m->field[s][c] : nullptr);
    for (int c = 0; c < 3 && !r; c++) r = field(b->J[c], m ? m->current[0][c] : nullptr);
    b->J0 = b->J[0];
    if (sheared(d))
        for (int c = 0; c < 3 && !r; c++) r = field(b->Jt[c], m ? m->current[1][c] : nullptr);
    for (int s = 0; s < b->nsp && !r; s++) {
        Species& S = b->sp[s];
        S.cap = d->capacity[s];
        S.qm = d->q_over_m[s];
        S.q = d->q_macro[s];
        const size_t cap = (size_t)S.cap + 1;
        for (int k = 0; k < 2 && !r; k++) {
            r = caller_buf(S.cell[k], m ? m->cell[s][k] : nullptr, cap);
            for (int c = 0; c < 3 && !r; c++) {
                if (c < b->dim)
                    r = caller_buf(S.off[k][c], m ? m->off[s][k][c] : nullptr, cap);
                else if (!m)
                    r = dalloc(b, S.off[k][c], 1);
            }
            for (int c = 0; c < 3 && !r; c++) r = caller_buf(S.u[k][c], m ? m->u[s][k][c] : nullptr, cap);
            if (!r && b->track_ids) r = caller_buf(S.id[k], m ? m->id[s][k] : nullptr, cap);
            if (escapes(d) && d->leaky_mode == PIC_LEAKY_DISPLACEMENT)
                for (int c = 0; c < 3 && !r; c++) r = caller_buf(S.dr[k][c], m ? m->dr[s][k][c] : nullptr, cap);
        }
        for (int k = 0; k < 2 && !r; k++) {
            r = dalloc(b, S.sb.keys[k], cap);
            if (!r) r = dalloc(b, S.sb.vals[k], cap);
        }
        if (!r) r = dalloc(b, S.sb.hist, sort_hist_words((int64_t)cap));
        if (!r) r = dalloc(b, S.sb.scratch, scan_scratch_words((int64_t)sort_hist_words((int64_t)cap)));
        for (int k = 0; k < 2 && !r; k++) r = dalloc(b, S.toff[k], (size_t)tiles_ws + 2);
        const size_t nt = (size_t)tiles_ws;
        if (!r) r = dalloc(b, S.sb.mcnt, nt * kMigDirs);
        if (!r) r = dalloc(b, S.sb.mpre, nt * kMigDirs);
        if (!r) r = dalloc(b, S.sb.tot, nt + 1);
        if (!r) r = dalloc(b, S.sb.start, nt + 1);
        if (!r) r = dalloc(b, S.sb.dcnt, nt + 1);
        if (!r) r = dalloc(b, S.sb.dpre, nt + 1);
        if (!r) r = dalloc(b, S.sb.mscratch, migrate_scratch_words(tiles_ws));
        if (!r) r = dalloc(b, S.sb.fallback, 1);
        if (!r) r = dalloc(b, S.n_live, 2);
        // the record of unfused pushes: reserved at creation on request (a box on caller
        // memory cannot take it later), else taken on first use
        if (!r && unfused_reserved(b)) {
            r = dalloc(b, S.ws_cell, cap);
            for (int c = 0; c < 3 && !r; c++) r = dalloc(b, S.ws_off[c], cap);
            for (int c = 0; c < 3 && !r; c++) r = dalloc(b, S.ws_disp[c], cap);
        }
        if (!r && !measuring && hipMemsetAsync(S.n_live, 0, 2 * sizeof(int32_t), b->st) != hipSuccess)
            r = PIC_EDEVICE;
    }
    if (!r) r = dalloc(b, b->err, 4);
    if (!r) r = dalloc(b, b->ctr, 4);
    if (!r && sheared(d)) r = dalloc(b, b->conv, kKsbConvWords);
    if (!r) r = dalloc(b, b->red_part, (size_t)10 * kRedBlocks);
    if (!r) r = dalloc(b, b->red_out, 16);
    if (!r) r = dalloc(b, b->hist_edges, kHistMaxBins + 1);
    if (!r) r = dalloc(b, b->hist_counts, kHistMaxBins + 2);
    if (!r && escapes(d) && d->leaky_mode == PIC_LEAKY_DISPLACEMENT)
        r = dalloc(b, b->mj, (size_t)kMjBins + kMjTail);
    if (measuring || r) return r;
    if (hipMemsetAsync(b->err, 0, 4 * sizeof(uint32_t), b->st) != hipSuccess) return PIC_EDEVICE;
    if (hipMemsetAsync(b->ctr, 0, 4 * sizeof(unsigned long long), b->st) != hipSuccess) return PIC_EDEVICE;
    if (b->conv && hipMemsetAsync(b->conv, 0, kKsbConvWords * sizeof(uint32_t), b->st) != hipSuccess)
        return PIC_EDEVICE;
    if (b->mj) {
        std::vector<float> tab;
        build_mj_table(d->leaky_theta_inj, tab);
        // synchronous copy from the host vector (it is freed on return)
        if (hipMemcpy(b->mj, tab.data(), tab.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
            return PIC_EDEVICE;
    }
    return PIC_OK;
}

// bytes of the arena: the workspace alone for a box on caller memory, everything otherwise
int32_t measure(pic_box* b, const pic_box_mem* m, size_t* bytes)
{
    b->alloc_pass = 1;
    b->arena_off = 0;
    const int32_t r = alloc_all(b, m);
    b->alloc_pass = 0;
    *bytes = b->arena_off;
    return r;
}

}  // namespace

// ================================================================ C ABI
extern "C" {

const char* pic_status_str(int32_t s)
{
    switch (s) {
    case PIC_OK: return "ok";
    case PIC_EINVAL: return "invalid argument";
    case PIC_ENOMEM: return "device allocation failed";
    case PIC_EDEVICE: return "HIP call failed";
    case PIC_ESTATE: return "call not valid in the current box state";
    case PIC_ECAP: return "particle count above capacity";
    default: return "unknown status";
    }
}

int32_t pic_device_copy(void* dst, const void* src, int64_t nbytes, void* stream)
{
    if (nbytes < 0 || (nbytes > 0 && (!dst || !src)) || (nbytes & 15) ||
        ((uintptr_t)dst & 15) || ((uintptr_t)src & 15))
        return PIC_EINVAL;
    return pic::device_copy16(dst, src, nbytes / 16, (hipStream_t)stream) == hipSuccess ? PIC_OK
                                                                                        : PIC_EDEVICE;
}

int32_t pic_box_destroy(pic_box* b)
{
    if (!b) return PIC_OK;
    hipStreamSynchronize(b->st);
    for (int s = 0; s < kMaxSpecies; s++) {
        if (b->side[s]) {
            hipStreamSynchronize(b->side[s]);
            hipStreamDestroy(b->side[s]);
        }
        if (b->side_ev[s]) hipEventDestroy(b->side_ev[s]);
    }
    if (b->fork_ev) hipEventDestroy(b->fork_ev);
    stager_release(b->stager);
    for (auto& a : b->allocs) lib_free(a.first, a.second);
    delete b;
    return PIC_OK;
}

int32_t pic_box_layout(const pic_box_desc* d, pic_box_layout_info* out)
{
    if (!d || !out) return PIC_EINVAL;
    pic_box* b = nullptr;
    int32_t r = init_box(d, nullptr, b);
    if (r) return r;
    std::memset(out, 0, sizeof(*out));
    pic_box_mem probe{};  // measuring with caller memory: the workspace alone
    size_t ws = 0;
    r = measure(b, &probe, &ws);
    if (!r) {
        out->workspace_bytes = (int64_t)ws;
        out->field_sets = b->nsets;
        out->current_arrays = sheared(d) ? 2 : 1;
        out->field_pitch_min[0] = b->G.sy;
        out->field_pitch_min[1] = b->G.sz;
        out->field_rows = (b->n[1] + 2 * b->G.g[1]) * (b->n[2] + 2 * b->G.g[2]);
        out->field_planes = b->n[2] + 2 * b->G.g[2];
        out->field_elems_min = b->comp_elems;
        for (int s = 0; s < b->nsp; s++) out->particle_elems[s] = d->capacity[s] + 1;
        out->has_id = b->track_ids ? 1 : 0;
        out->has_dr = escapes(d) && d->leaky_mode == PIC_LEAKY_DISPLACEMENT ? 1 : 0;
    }
    delete b;
    return r;
}

int32_t pic_workspace_bytes(const pic_box_desc* d, int64_t* bytes)
{
    if (!bytes) return PIC_EINVAL;
    pic_box_layout_info L{};
    const int32_t r = pic_box_layout(d, &L);
    if (!r) *bytes = L.workspace_bytes;
    return r;
}

int32_t pic_allocated_bytes(int64_t* device_bytes, int64_t* host_bytes)
{
    if (device_bytes) *device_bytes = g_dev_bytes.load();
    if (host_bytes) *host_bytes = g_host_bytes.load();
    return PIC_OK;
}

int32_t pic_box_create(const pic_box_desc* d, const pic_box_mem* m, pic_box** out)
{
    if (!d || !out) return PIC_EINVAL;
    pic_box* b = nullptr;
    int32_t r = init_box(d, m ? m->field_pitch : nullptr, b);
    if (r) return r;
    b->caller_mem = m != nullptr;
    size_t bytes = 0;
    r = measure(b, m, &bytes);
    if (!r && m) {
        // the caller's workspace: large enough and 256-byte aligned
        if (!m->workspace || m->workspace_bytes < (int64_t)bytes || (reinterpret_cast<uintptr_t>(m->workspace) & 255))
            r = m->workspace && m->workspace_bytes < (int64_t)bytes ? PIC_ENOMEM : PIC_EINVAL;
        else
            b->arena = static_cast<char*>(m->workspace);
    } else if (!r) {
        void* q = nullptr;
        if (lib_malloc(&q, bytes) != hipSuccess) {
            r = PIC_ENOMEM;
        } else {
            b->allocs.push_back({q, bytes});
            b->arena = static_cast<char*>(q);
        }
    }
    if (!r) {
        b->alloc_pass = 2;
        b->arena_off = 0;
        r = alloc_all(b, m);
        b->alloc_pass = 0;
    }
    if (r) {
        pic_box_destroy(b);
        return r;
    }
    *out = b;
    return PIC_OK;
}

int32_t pic_set_fields(pic_box* b, const float* E, const float* B)
{
    if (!b || !E || !B) return PIC_EINVAL;
    const int64_t nc = (int64_t)b->n[0] * b->n[1] * b->n[2];
    for (int c = 0; c < 3; c++) {
        if (interior_copy(b->G, b->E(c), const_cast<float*>(E) + c * nc, 0, b->st) != hipSuccess)
            return PIC_EDEVICE;
        if (interior_copy(b->G, b->B(c), const_cast<float*>(B) + c * nc, 0, b->st) != hipSuccess)
            return PIC_EDEVICE;
    }
    return fill_field_guards(b, time_of(b, b->step));
}

int32_t pic_get_fields(pic_box* b, float* E, float* B)
{
    if (!b) return PIC_EINVAL;
    const int64_t nc = (int64_t)b->n[0] * b->n[1] * b->n[2];
    for (int c = 0; c < 3; c++) {
        if (E && interior_copy(b->G, b->E(c), E + c * nc, 1, b->st) != hipSuccess) return PIC_EDEVICE;
        if (B && interior_copy(b->G, b->B(c), B + c * nc, 1, b->st) != hipSuccess) return PIC_EDEVICE;
    }
    return hip_fail(hipStreamSynchronize(b->st));
}

int32_t pic_get_current(pic_box* b, float* J)
{
    if (!b || !J) return PIC_EINVAL;
    const int64_t nc = (int64_t)b->n[0] * b->n[1] * b->n[2];
    for (int c = 0; c < 3; c++)
        if (interior_copy(b->G, b->J[c], J + c * nc, 1, b->st) != hipSuccess) return PIC_EDEVICE;
    return hip_fail(hipStreamSynchronize(b->st));
}

int32_t pic_set_particles(pic_box* b, int32_t s, int64_t n, const int32_t* cell, const float* off,
                          const float* u, const uint32_t* id, const float* dr)
{
    if (!b || s < 0 || s >= b->nsp || n < 0 || (n > 0 && (!cell || !off || !u))) return PIC_EINVAL;
    if (side_join(b)) return PIC_EDEVICE;
    Species& S = b->sp[s];
    if (n > S.cap) return PIC_ECAP;
    hipStream_t st = b->st;
    const int k = S.cur;
    if (cells_linear_to_packed(cell, S.cell[k], n, b->n, b->cc, b->err, st) != hipSuccess) return PIC_EDEVICE;
    const size_t fb = sizeof(float) * (size_t)n;
    for (int c = 0; c < b->dim; c++)
        if (n && hipMemcpyAsync(S.off[k][c], off + c * n, fb, hipMemcpyDeviceToDevice, st) != hipSuccess)
            return PIC_EDEVICE;
    for (int c = 0; c < 3; c++)
        if (n && hipMemcpyAsync(S.u[k][c], u + c * n, fb, hipMemcpyDeviceToDevice, st) != hipSuccess)
            return PIC_EDEVICE;
    if (b->track_ids) {
        if (id) {
            if (n && hipMemcpyAsync(S.id[k], id, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, st) != hipSuccess)
                return PIC_EDEVICE;
        } else if (iota_u32(S.id[k], n, st) != hipSuccess) {
            return PIC_EDEVICE;
        }
    }
    if (S.dr[k][0]) {
        for (int c = 0; c < 3; c++) {
            if (dr) {
                if (n && hipMemcpyAsync(S.dr[k][c], dr + c * n, fb, hipMemcpyDeviceToDevice, st) != hipSuccess)
                    return PIC_EDEVICE;
            } else if (zero_floats(S.dr[k][c], n, st) != hipSuccess) {
                return PIC_EDEVICE;
            }
        }
    }
    if (set_i32(S.n_live, (int32_t)n, st) != hipSuccess) return PIC_EDEVICE;
    b->record_valid = false;
    S.n_upper = (int)n;
    S.grouped = false;
    S.counts_ready = false;
    b->sorted = false;
    return PIC_OK;
}

int32_t pic_get_particles(pic_box* b, int32_t s, int64_t* n_out, int32_t* cell, float* off, float* u,
                          uint32_t* id, float* dr)
{
    if (!b || s < 0 || s >= b->nsp) return PIC_EINVAL;
    if (side_join(b)) return PIC_EDEVICE;
    Species& S = b->sp[s];
    int32_t n = 0;
    if (hipMemcpyAsync(&n, S.n_live, sizeof(int32_t), hipMemcpyDeviceToHost, b->st) != hipSuccess ||
        hipStreamSynchronize(b->st) != hipSuccess)
        return PIC_EDEVICE;
    if (n_out) *n_out = n;
    const int k = S.cur;
    hipStream_t st = b->st;
    const size_t fb = sizeof(float) * (size_t)n;
    if (cell && cells_packed_to_linear(S.cell[k], cell, n, b->n, b->cc, st) != hipSuccess) return PIC_EDEVICE;
    for (int c = 0; c < b->dim && off; c++)
        if (n && hipMemcpyAsync(off + c * n, S.off[k][c], fb, hipMemcpyDeviceToDevice, st) != hipSuccess)
            return PIC_EDEVICE;
    for (int c = 0; c < 3 && u; c++)
        if (n && hipMemcpyAsync(u + c * n, S.u[k][c], fb, hipMemcpyDeviceToDevice, st) != hipSuccess)
            return PIC_EDEVICE;
    if (id && b->track_ids && n &&
        hipMemcpyAsync(id, S.id[k], sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return PIC_EDEVICE;
    // the z displacement is tracked only with the 3-vector escape test: 0 otherwise
    const int ndr = b->d.leaky_use_3vec ? 3 : 2;
    for (int c = 0; c < ndr && dr && S.dr[k][0]; c++)
        if (n && hipMemcpyAsync(dr + c * n, S.dr[k][c], fb, hipMemcpyDeviceToDevice, st) != hipSuccess)
            return PIC_EDEVICE;
    if (dr && S.dr[k][0] && ndr == 2 && zero_floats(dr + 2 * n, n, st) != hipSuccess) return PIC_EDEVICE;
    return hip_fail(hipStreamSynchronize(st));
}

int32_t pic_get_sort(pic_box* b, int32_t s, int32_t* perm, int32_t* offsets, int32_t* n_tiles_out)
{
    if (!b || s < 0 || s >= b->nsp) return PIC_EINVAL;
    if (side_join(b)) return PIC_EDEVICE;
    Species& S = b->sp[s];
    if (n_tiles_out) *n_tiles_out = b->tl.n_tiles;
    int32_t n = 0;
    const int32_t* toff = S.toff[S.toff_cur];
    if (hipMemcpyAsync(&n, toff + b->tl.n_tiles, sizeof(int32_t), hipMemcpyDeviceToHost, b->st) != hipSuccess ||
        hipStreamSynchronize(b->st) != hipSuccess)
        return PIC_EDEVICE;
    if (perm && n &&
        hipMemcpyAsync(perm, S.sb.vals[S.which], sizeof(int32_t) * n, hipMemcpyDeviceToDevice, b->st) != hipSuccess)
        return PIC_EDEVICE;
    if (offsets && hipMemcpyAsync(offsets, toff, sizeof(int32_t) * (b->tl.n_tiles + 1),
                                  hipMemcpyDeviceToDevice, b->st) != hipSuccess)
        return PIC_EDEVICE;
    return hip_fail(hipStreamSynchronize(b->st));
}

int32_t pic_get_push_record(pic_box* b, int32_t s, int64_t* n_out, int32_t* cell, float* off,
                            float* disp)
{
    if (!b || s < 0 || s >= b->nsp) return PIC_EINVAL;
    if (side_join(b)) return PIC_EDEVICE;
    if (!b->record_valid) return PIC_ESTATE;
    Species& S = b->sp[s];
    int32_t n = 0;
    if (hipMemcpyAsync(&n, S.n_live, sizeof(int32_t), hipMemcpyDeviceToHost, b->st) != hipSuccess ||
        hipStreamSynchronize(b->st) != hipSuccess)
        return PIC_EDEVICE;
    if (n_out) *n_out = n;
    hipStream_t st = b->st;
    const size_t fb = sizeof(float) * (size_t)n;
    if (cell && cells_packed_to_linear(S.ws_cell, cell, n, b->n, b->cc, st) != hipSuccess) return PIC_EDEVICE;
    for (int c = 0; c < b->dim && off; c++)
        if (n && hipMemcpyAsync(off + c * n, S.ws_off[c], fb, hipMemcpyDeviceToDevice, st) != hipSuccess)
            return PIC_EDEVICE;
    for (int c = 0; c < 3 && disp; c++)
        if (n && hipMemcpyAsync(disp + c * n, S.ws_disp[c], fb, hipMemcpyDeviceToDevice, st) != hipSuccess)
            return PIC_EDEVICE;
    return hip_fail(hipStreamSynchronize(st));
}

int32_t pic_tile_sort(pic_box* const* boxes, int32_t nb, uint32_t flags)
{
    int32_t r = check_boxes(boxes, nb);
    for (int i = 0; i < nb && !r; i++) {
        pic_box* b = boxes[i];
        if (!(flags & PIC_SORT_OVERLAP)) {
            r = sort_box(b);
            continue;
        }
        // fork: each species' side stream takes over after the work queued so far (the push
        // that wrote the positions); the species' sorts run there, side by side; the join is
        // left to the next call that touches particles or the sort
        if (b->deposit_pending) return PIC_ESTATE;
        if (side_join(b)) return PIC_EDEVICE;
        // created on first use (each that is still missing, so a failed creation is retried)
        if (!b->fork_ev && hipEventCreateWithFlags(&b->fork_ev, hipEventDisableTiming) != hipSuccess)
            return PIC_EDEVICE;
        for (int s = 0; s < b->nsp; s++)
            if ((!b->side[s] && hipStreamCreateWithFlags(&b->side[s], hipStreamNonBlocking) != hipSuccess) ||
                (!b->side_ev[s] && hipEventCreateWithFlags(&b->side_ev[s], hipEventDisableTiming) != hipSuccess))
                return PIC_EDEVICE;
        if (hipEventRecord(b->fork_ev, b->st) != hipSuccess) return PIC_EDEVICE;
        for (int s = 0; s < b->nsp; s++) {
            if (hipStreamWaitEvent(b->side[s], b->fork_ev, 0) != hipSuccess ||
                sort_species(b, s, b->side[s]) != PIC_OK || hipEventRecord(b->side_ev[s], b->side[s]) != hipSuccess)
                return PIC_EDEVICE;
        }
        b->sorted = true;
        b->side_pending = true;
    }
    return r;
}

int32_t pic_gather_push(pic_box* const* boxes, int32_t nb, uint32_t flags)
{
    int32_t r = check_boxes(boxes, nb);
    for (int i = 0; i < nb && !r; i++) r = push_box(boxes[i], (flags & PIC_FUSE_DEPOSIT) != 0);
    return r;
}

int32_t pic_deposit(pic_box* const* boxes, int32_t nb, uint32_t)
{
    int32_t r = check_boxes(boxes, nb);
    for (int i = 0; i < nb && !r; i++) r = deposit_box(boxes[i]);
    return r;
}

int32_t pic_shear_remap(pic_box* const* boxes, int32_t nb, uint32_t what)
{
    int32_t r = check_boxes(boxes, nb);
    for (int i = 0; i < nb && !r; i++) {
        pic_box* b = boxes[i];
        if (what & PIC_REMAP_CURRENT) r = fold_box(b);
        if (!r && (what & PIC_REMAP_FIELDS)) r = fill_field_guards(b, time_of(b, b->step));
    }
    return r;
}

int32_t pic_maxwell_step(pic_box* const* boxes, int32_t nb, uint32_t)
{
    int32_t r = check_boxes(boxes, nb);
    for (int i = 0; i < nb && !r; i++) {
        pic_box* b = boxes[i];
        r = maxwell_box(b);
        if (!r) {
            b->step += 1;
            if (!sheared(&b->d)) r = fill_field_guards(b, time_of(b, b->step));
        }
    }
    return r;
}

int32_t pic_escape_compact(pic_box* const* boxes, int32_t nb, uint32_t flags)
{
    return pic_tile_sort(boxes, nb, flags);
}

int32_t pic_tile_candidates(int32_t dim, uint32_t flags, int32_t* shapes_out, int32_t max_out)
{
    if ((dim != 2 && dim != 3) || max_out < 0 || (max_out > 0 && !shapes_out)) return PIC_EINVAL;
    int c[8][3];
    const int n = tile_candidates(dim, (flags & PIC_TUNE_BATCHED) != 0, c, 8);
    for (int i = 0; i < n && i < max_out; i++)
        for (int k = 0; k < 3; k++) shapes_out[3 * i + k] = c[i][k];
    return n;
}

int32_t pic_autotune(pic_box* b, uint32_t flags, int32_t trials, int32_t* tile_out, float* ms_out,
                     int32_t max_out, int32_t* n_out)
{
    if (!b || !tile_out || trials < 1 || trials > 64) return PIC_EINVAL;
    if (side_join(b)) return PIC_EDEVICE;
    if (b->deposit_pending) return PIC_ESTATE;
    int64_t live = 0;
    for (int s = 0; s < b->nsp; s++) live += b->sp[s].n_upper;
    if (live == 0) return PIC_ESTATE;  // nothing to time
    int cand[8][3];
    const int nc = tile_candidates(b->dim, (flags & PIC_TUNE_BATCHED) != 0, cand, 8);
    hipStream_t st = b->st;
    // the trials leave nothing the caller sees: error bits, counters and the slot counts the
    // next sort starts from are restored after
    uint32_t err[4];
    unsigned long long ctr[4];
    int32_t nlive[kMaxSpecies][2];
    if (hipStreamSynchronize(st) != hipSuccess ||
        hipMemcpy(err, b->err, sizeof err, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(ctr, b->ctr, sizeof ctr, hipMemcpyDeviceToHost) != hipSuccess)
        return PIC_EDEVICE;
    for (int s = 0; s < b->nsp; s++)
        if (hipMemcpy(nlive[s], b->sp[s].n_live, sizeof nlive[s], hipMemcpyDeviceToHost) != hipSuccess)
            return PIC_EDEVICE;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return PIC_EDEVICE;
    const int tile0[3] = {b->tile[0], b->tile[1], b->tile[2]};
    int32_t r = PIC_OK;
    float best_ms = 0.f;
    int best = -1;
    bool best_mig = false;
    for (int i = 0; i < nc && !r; i++) {
        set_tiling(b, cand[i]);
        float ms = 0.f;
        // each trial: a fresh radix sort in this tiling, then the fused push into the spare
        // particle buffers and the current array (the box state is not advanced); the first
        // trial warms up, the fastest of the others counts
        for (int t = 0; t <= trials && !r; t++) {
            for (int s = 0; s < b->nsp; s++) b->sp[s].grouped = false;
            r = sort_box(b);
            if (!r) r = zero_current(b);
            if (r) break;
            const StepDev P = make_step(b);
            if (hipEventRecord(e0, st) != hipSuccess ||
                launch_gather_push(P, b->tile, 1, st) != hipSuccess ||
                hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                r = PIC_EDEVICE;
                break;
            }
            float m = 0.f;
            if (hipEventElapsedTime(&m, e0, e1) != hipSuccess) r = PIC_EDEVICE;
            if (t == 1 || (t > 1 && m < ms)) ms = m;
        }
        if (r) break;
        if (ms_out && i < max_out) ms_out[i] = ms;
        // a tiling that admits the migration sort wins over one that does not (the sort after
        // every push is then a counting sort over neighbouring tiles instead of a radix sort)
        if (best < 0 || (b->mig_ok && !best_mig) || (b->mig_ok == best_mig && ms < best_ms)) {
            best = i;
            best_ms = ms;
            best_mig = b->mig_ok;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    set_tiling(b, r ? tile0 : cand[best]);
    for (int s = 0; s < b->nsp; s++) b->sp[s].grouped = b->sp[s].counts_ready = false;
    b->sorted = false;
    if (hipStreamSynchronize(st) != hipSuccess ||
        hipMemcpy(b->err, err, sizeof err, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->ctr, ctr, sizeof ctr, hipMemcpyHostToDevice) != hipSuccess)
        r = r ? r : PIC_EDEVICE;
    for (int s = 0; s < b->nsp; s++)
        if (hipMemcpy(b->sp[s].n_live, nlive[s], sizeof nlive[s], hipMemcpyHostToDevice) != hipSuccess)
            r = r ? r : PIC_EDEVICE;
    if (r) return r;
    for (int k = 0; k < 3; k++) tile_out[k] = b->tile[k];
    if (n_out) *n_out = nc;
    return PIC_OK;
}

int32_t pic_step(pic_box* const* boxes, int32_t nb, uint32_t flags)
{
    int32_t r = check_boxes(boxes, nb);
    for (int i = 0; i < nb && !r; i++) r = side_join(boxes[i]);
    if (!r && (flags & (PIC_STEP_BATCHED | PIC_STEP_GRAPH))) {
        // the lead box stages the tables in its own (library) memory; a box on caller memory
        // cannot, and leads batched steps only through pic_step_batch
        if (boxes[0]->caller_mem) return PIC_EINVAL;
        return step_batched(boxes, nb, (flags & PIC_STEP_GRAPH) != 0, boxes[0]->stager, false, nullptr);
    }
    for (int i = 0; i < nb && !r; i++) {
        pic_box* b = boxes[i];
        r = sort_box(b);
        if (!r) r = push_box(b, true);
        if (!r) r = fold_box(b);
        if (!r) r = maxwell_box(b);
        if (!r) {
            b->step += 1;
            if (!sheared(&b->d)) r = fill_field_guards(b, time_of(b, b->step));
        }
    }
    return r;
}

int32_t pic_batch_create(void* dev, void* host, int64_t bytes, void* stream, pic_batch** out)
{
    if (!out || !dev || !host || bytes < 2 * 4096 || (reinterpret_cast<uintptr_t>(dev) & 255) ||
        (reinterpret_cast<uintptr_t>(host) & 255))
        return PIC_EINVAL;
    pic_batch* B = new (std::nothrow) pic_batch();
    if (!B) return PIC_ENOMEM;
    B->st = static_cast<hipStream_t>(stream);
    B->sg.caller = true;
    const size_t half = ((size_t)bytes / 2) & ~(size_t)255;
    for (int k = 0; k < 2; k++) {
        B->sg.buf[k].dev = static_cast<char*>(dev) + k * half;
        B->sg.buf[k].host = static_cast<char*>(host) + k * half;
        B->sg.buf[k].cap = half;
    }
    *out = B;
    return PIC_OK;
}

int32_t pic_batch_destroy(pic_batch* B)
{
    if (!B) return PIC_OK;
    hipStreamSynchronize(B->st);
    stager_release(B->sg);
    delete B;
    return PIC_OK;
}

int32_t pic_step_batch(pic_batch* B, pic_box* const* boxes, int32_t nb, uint32_t flags)
{
    if (!B) return PIC_EINVAL;
    int32_t r = check_boxes(boxes, nb);
    for (int i = 0; i < nb && !r; i++)
        if (boxes[i]->st != B->st) r = PIC_EINVAL;
    for (int i = 0; i < nb && !r; i++) r = side_join(boxes[i]);
    if (r) return r;
    return step_batched(boxes, nb, (flags & PIC_STEP_GRAPH) != 0, B->sg, false, nullptr);
}

int32_t pic_step_table_bytes(pic_box* const* boxes, int32_t nb, int64_t* bytes)
{
    if (!bytes) return PIC_EINVAL;
    int32_t r = check_boxes(boxes, nb);
    if (r) return r;
    Stager unused;
    size_t tb = 0;
    r = step_batched(boxes, nb, false, unused, true, &tb);
    if (!r) *bytes = (int64_t)tb;
    return r;
}

int32_t pic_set_step(pic_box* b, int64_t step)
{
    if (!b || step < 0) return PIC_EINVAL;
    if (b->deposit_pending) return PIC_ESTATE;
    b->step = step;
    return fill_field_guards(b, time_of(b, step));
}

int32_t pic_energy_histogram(pic_box* b, int32_t s, const double* edges, int32_t nbins, uint64_t* counts)
{
    if (!b || s < 0 || s >= b->nsp || !edges || !counts || nbins < 1 || nbins > kHistMaxBins)
        return PIC_EINVAL;
    if (side_join(b)) return PIC_EDEVICE;
    for (int i = 0; i <= nbins; i++)
        if (!std::isfinite(edges[i]) || (i > 0 && !(edges[i] > edges[i - 1]))) return PIC_EINVAL;
    static_assert(PIC_HIST_MAX_BINS == kHistMaxBins, "histogram size");
    hipStream_t st = b->st;
    const Species& S = b->sp[s];
    const int k = S.cur;
    if (hipMemcpyAsync(b->hist_edges, edges, sizeof(double) * (nbins + 1), hipMemcpyHostToDevice, st) !=
            hipSuccess ||
        energy_histogram(S.cell[k], S.u[k][0], S.u[k][1], S.u[k][2], S.n_live, b->hist_edges, nbins,
                         b->hist_counts, kRedBlocks, st) != hipSuccess ||
        hipMemcpyAsync(counts, b->hist_counts, sizeof(uint64_t) * (nbins + 2), hipMemcpyDeviceToHost, st) !=
            hipSuccess)
        return PIC_EDEVICE;
    return hip_fail(hipStreamSynchronize(st));
}

int32_t pic_energy_histogram_static(pic_box* b, int32_t s, const double* edges, int32_t nbins,
                                    uint64_t* counts)
{
    if (!b || s < 0 || s >= b->nsp || !edges || !counts || nbins < 1) return PIC_EINVAL;
    if (nbins > PIC_HIST_STATIC_MAX_BINS) return PIC_EINVAL;  // beyond the static scratch
    if (side_join(b)) return PIC_EDEVICE;
    for (int i = 0; i <= nbins; i++)
        if (!std::isfinite(edges[i]) || (i > 0 && !(edges[i] > edges[i - 1]))) return PIC_EINVAL;
    static_assert(PIC_HIST_STATIC_MAX_BINS <= kHistMaxBins, "static histogram size");
    void* scr = nullptr;
    size_t scr_bytes = 0;
    if (static_scratch(&scr, &scr_bytes) != hipSuccess) return PIC_EDEVICE;
    if (scr_bytes < kStaticHistCountsOffset + sizeof(uint64_t) * (size_t)(nbins + 2)) return PIC_EINVAL;
    double* dev_edges = static_cast<double*>(scr);
    auto* dev_counts = reinterpret_cast<unsigned long long*>(static_cast<char*>(scr) + kStaticHistCountsOffset);
    hipStream_t st = b->st;
    const Species& S = b->sp[s];
    const int k = S.cur;
    // energy_histogram clears the counts with a fill kernel before it adds into them (the
    // scratch keeps the last call's contents)
    if (hipMemcpyAsync(dev_edges, edges, sizeof(double) * (nbins + 1), hipMemcpyHostToDevice, st) !=
            hipSuccess ||
        energy_histogram(S.cell[k], S.u[k][0], S.u[k][1], S.u[k][2], S.n_live, dev_edges, nbins,
                         dev_counts, kRedBlocks, st) != hipSuccess ||
        hipMemcpyAsync(counts, dev_counts, sizeof(uint64_t) * (nbins + 2), hipMemcpyDeviceToHost, st) !=
            hipSuccess)
        return PIC_EDEVICE;
    return hip_fail(hipStreamSynchronize(st));
}

int32_t pic_box_get(pic_box* b, pic_box_info* info)
{
    if (!b || !info) return PIC_EINVAL;
    if (side_join(b)) return PIC_EDEVICE;
    std::memset(info, 0, sizeof(*info));
    hipStream_t st = b->st;
    if (field_energy(b->G, field_ptrs(b), 6, b->red_part, kRedBlocks, b->red_out, st) != hipSuccess)
        return PIC_EDEVICE;
    double fe[6];
    if (hipMemcpyAsync(fe, b->red_out, sizeof(fe), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return PIC_EDEVICE;
    for (int c = 0; c < 3; c++) {
        info->field_energy_B[c] = fe[c] / (8.0 * kPi);  // set order: B then E
        info->field_energy_E[c] = fe[3 + c] / (8.0 * kPi);
    }
    for (int s = 0; s < b->nsp; s++) {
        Species& S = b->sp[s];
        const int k = S.cur;
        if (particle_sums(S.cell[k], S.u[k][0], S.u[k][1], S.u[k][2], S.n_live, b->red_part, kRedBlocks,
                          b->red_out, st) != hipSuccess)
            return PIC_EDEVICE;
        double ps[kPartSums];
        int32_t n = 0;
        if (hipMemcpyAsync(ps, b->red_out, sizeof(ps), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipMemcpyAsync(&n, S.n_live, sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return PIC_EDEVICE;
        const double m = S.qm != 0 ? std::fabs(S.q / S.qm) : 0.0;
        info->kinetic_energy += m * ps[0];
        for (int c = 0; c < 3; c++) info->momentum[c] += m * ps[1 + c];
        for (int c = 0; c < 3; c++) info->pressure[c] += m * ps[4 + c];
        info->n_particles[s] = n;
    }
    uint32_t err = 0;
    unsigned long long ctr[4] = {0, 0, 0, 0};
    if (hipMemcpy(&err, b->err, sizeof(err), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(ctr, b->ctr, sizeof(ctr), hipMemcpyDeviceToHost) != hipSuccess)
        return PIC_EDEVICE;
    info->maxwell_sweeps = b->last_sweeps;
    if (b->last_sweeps < 0 &&
        hipMemcpy(&info->maxwell_sweeps, b->conv + 2 * kKsbMaxSweeps, sizeof(int32_t), hipMemcpyDeviceToHost) !=
            hipSuccess)
        return PIC_EDEVICE;
    info->n_sort_migrations = b->n_migrations;
    info->n_sort_fallbacks = (int64_t)ctr[2];
    info->errors = err;
    info->n_slow = (int64_t)ctr[0];
    info->n_escaped = (int64_t)ctr[1];
    info->n_superluminal = (int64_t)ctr[3];
    info->field_set = b->cur_set;
    info->current_array = b->J[0] == b->J0 ? 0 : 1;
    for (int s = 0; s < b->nsp; s++) info->particle_copy[s] = b->sp[s].cur;
    info->step = b->step;
    info->t = time_of(b, b->step);
    info->dys = shear_offset(b, info->t);
    info->a = 1.0;
    for (int k = 0; k < 3; k++)
        if (expanding(&b->d) && ((b->d.expand_axis_mask >> k) & 1)) info->a = scale_of(b, k, info->t);
    return PIC_OK;
}

}  // extern "C"
