/*
 * pic.h — C ABI of the MI355X particle hot path for the extended particle-in-cell
 * methods of Bacchini et al., "Particle-in-Cell Methods for Simulations of Sheared,
 * Expanding, or Escaping Astrophysical Plasma" (arXiv 2602.15939):
 *   the shearing box with orbital advection (Sec. 2), the expanding box (Sec. 3)
 *   and the leaky box (Sec. 4), on a Yee grid with charge-conserving deposition.
 *
 * Conventions (every call):
 *   - code units: c = 1, cell size dx = 1, Gaussian units with an explicit 4*pi;
 *   - return value: PIC_OK (0) or a negative pic_status; nothing throws or aborts;
 *   - all device work is asynchronous on the box stream (desc.stream, a hipStream_t;
 *     NULL = the null stream) unless the call says it synchronises;
 *   - device memory: a box is created either on caller-owned memory (pic_box_mem: the
 *     particle arrays, the field and current arrays and one workspace block, e.g. torch
 *     tensors; the library then never allocates for that box) or, with no pic_box_mem, on
 *     memory the library allocates and frees with the box.  Other pointers passed in or out
 *     are caller-owned; a pointer argument named *_dev must be device memory, *_host host
 *     memory;
 *   - handles are not thread-safe; calls on one box must not overlap;
 *   - fields are stored as the frame's evolved variables: E' and B for the shearing box
 *     (Sec. 2.1), lab-frame E and B at the primed coordinates for the expanding box
 *     (Sec. 3.2), E and B otherwise;
 *   - grid layout at the boundary: one component array holds n[0]*n[1]*n[2] floats,
 *     x fastest; the Yee offsets (cells) are Ex(1/2,0,0) Ey(0,1/2,0) Ez(0,0,1/2),
 *     Bx(0,1/2,1/2) By(1/2,0,1/2) Bz(1/2,1/2,0), J as E; in 2D n[2] = 1;
 *   - particle layout at the boundary (structure of arrays): cell[n] int32 linear cell
 *     index i + n0*(j + n1*k); off[dim][n] float in-cell offsets in [0,1); u[3][n] float
 *     spatial part of the four-velocity (u' in the shearing box, Sec. 2.1); id[n] uint32;
 *     dr[3][n] float leaky-box displacement (Sec. 4.1; dr[2] is tracked only with
 *     leaky_use_3vec and reads back as 0 otherwise).
 */
#ifndef PIC_H
#define PIC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum pic_status {
    PIC_OK = 0,
    PIC_EINVAL = -1,  /* invalid argument (unsupported combination, CFL, null pointer) */
    PIC_ENOMEM = -2,  /* device allocation failed */
    PIC_EDEVICE = -3, /* a HIP call failed */
    PIC_ESTATE = -4,  /* call not valid in the box's current state */
    PIC_ECAP = -5     /* particle count above the species capacity */
} pic_status;

enum pic_frame { PIC_FRAME_PLAIN = 0, PIC_FRAME_SHEAR = 1, PIC_FRAME_EXPAND = 2, PIC_FRAME_LEAKY = 3,
                 PIC_FRAME_SHEAR_EXPAND = 4 };
/* PIC_FRAME_SHEAR_EXPAND: the shearing box of Sec. 2 in the expanding coordinates of Sec. 3 (the
   combination the conclusion, Sec. 5, names).  The push solves eq. OAu_disc with the Lambda of
   eq. EBu_disc added (Sherman-Morrison of the rank-1 S around the printed B^(Lambda) inverse),
   positions move by dt L^-1 u'/gamma' plus the shear move, and the field step is the implicit
   midpoint of Sec. 2.2 on the expanding-frame fields (l/l_c) F_c with the (1/l) L^2 curl factors
   of eqs. EBB/EBE.  x and y scale together: expand_axis_mask 0, 4 (z), 3 (xy) or 7; other masks
   are PIC_EINVAL.  The field step takes the one-thread-per-cell sweeps (also in a batched
   step, where the conversions to and from the expanding-frame fields are batched launches). */
enum pic_leaky_mode { PIC_LEAKY_DISPLACEMENT = 0, PIC_LEAKY_PROBABILISTIC = 1 };

/* pic_gather_push flags */
#define PIC_FUSE_DEPOSIT 1u /* deposit the current inside the push kernel (the hot path) */
/* pic_shear_remap selection */
#define PIC_REMAP_FIELDS 1u
#define PIC_REMAP_CURRENT 2u
/* pic_step flags */
#define PIC_STEP_BATCHED 1u /* one launch per kernel for all boxes (box-descriptor tables) */
#define PIC_STEP_GRAPH 2u   /* the batched step as a captured HIP graph, replayed while the box
                               set and its launch shapes stay the same (implies BATCHED) */
/* pic_tile_sort flags */
#define PIC_SORT_OVERLAP 1u /* run the sort of each species on a stream of its own (the species'
                               sorts side by side), after the work queued on the box stream so
                               far (the push that wrote the positions), so that it overlaps the
                               current fold and the Maxwell step queued after it; the next call that reads or writes particles or the sort
                               (push, deposit, sort, escape compaction, particle and sort copies,
                               pic_box_get, pic_step, pic_autotune, the histogram) first waits for
                               it; pic_shear_remap, pic_maxwell_step and the field and current
                               calls do not */
/* pic_autotune flags */
#define PIC_TUNE_BATCHED 1u /* only the tile shapes the batched step supports */
/* pic_box_desc.flags */
#define PIC_BOX_TRACK_IDS 1u /* carry particle ids through the sort (always on for LEAKY) */
#define PIC_BOX_COUNT_SUPERLUMINAL 2u /* shearing box: count pushes whose effective velocity
                                         exceeds c (pic_box_info.n_superluminal); ~2 % of the
                                         fused kernel's time, so off unless asked for */
#define PIC_BOX_ESCAPE 4u    /* apply the leaky box's escape rule (leaky_mode and its
                                parameters, Sec. 4.1) in the shearing or expanding frame too,
                                the combination the conclusion of the paper suggests; the
                                displacement is the one the deposit uses: comoving (x' - x^n,
                                relative to the shear flow) or primed (expanding box); ids are
                                carried.  Implied by PIC_FRAME_LEAKY */
#define PIC_BOX_UNFUSED 8u   /* reserve at creation the record of unfused pushes (28 B per
                                particle of capacity: old position and deposit displacement) that
                                pic_gather_push without PIC_FUSE_DEPOSIT, pic_deposit and
                                pic_get_push_record use.  A box on caller memory needs it for
                                them (PIC_ESTATE otherwise); a library-owned box without it
                                allocates the record on the first unfused push */

/* sticky device error bits (pic_box_info.errors) */
#define PIC_DERR_CFL 1u      /* a deposit displacement reached half a cell, or (shearing box)
                                the y increment with the shear move reached a whole cell */
#define PIC_DERR_NAN 2u      /* non-finite momentum */
#define PIC_DERR_ORDER 4u    /* a particle outside its tile: handled on the slow path */
#define PIC_DERR_CELL 8u     /* pic_set_particles met a cell index outside the grid */
#define PIC_DERR_SORT 16u    /* a batched sort found a particle beyond the neighbouring tiles */
#define PIC_DERR_NOCONVERGE 32u /* shearing box, maxwell_tol > 0: the fixed-point sweeps of a
                                   Maxwell step did not meet the tolerance within maxwell_iters */

typedef struct pic_box_desc {
    int32_t dim;         /* 2 or 3 */
    int32_t n[3];        /* cells per axis (n[2] = 1 in 2D); n[0]*n[1]*n[2] < 2^31 */
    double dt;           /* time step; requires dt*sqrt(dim) < 1 (Yee CFL) */
    int32_t frame;       /* enum pic_frame */
    /* shearing box (Sec. 2.1): v_s = -s*Omega0*x e_y, x = X - n[0]/2 */
    double shear_s, shear_omega0;
    /* expanding box (Sec. 3.1): l_d(t) = 1 + expand_adot*t on the axes in expand_axis_mask */
    double expand_adot;
    int32_t expand_axis_mask;
    /* leaky box (Sec. 4.1) */
    int32_t leaky_mode;      /* enum pic_leaky_mode */
    double leaky_l_esc;      /* displacement mode: escape distance */
    int32_t leaky_use_3vec;  /* displacement mode: test (dx, dy, dz) instead of (dx, dy);
                                dz is tracked only then */
    double leaky_theta_inj;  /* displacement mode: Maxwell-Juttner temperature of reinjection */
    double leaky_t_esc;      /* probabilistic mode: escape probability dt/t_esc per step ... */
    double leaky_gamma_thr;  /* ... for particles with gamma > gamma_thr */
    /* species */
    int32_t n_species;       /* 1 or 2 */
    double q_over_m[2];      /* charge-to-mass ratio (sign included) */
    double q_macro[2];       /* macro-particle charge (sign included) */
    int64_t capacity[2];     /* maximum particle count per species (below 2^30) */
    uint64_t seed;           /* Philox4x32-10 key */
    uint32_t box_id;         /* fourth Philox counter word */
    int32_t tile[3];         /* tile shape in cells (0 = default: 8^3 in 3D, 16x16 in 2D;
                                supported: 8^3, 4^3; 16x16, 8x8, 32x16, 32x32); pic_autotune
                                picks one by measurement */
    int32_t maxwell_iters;   /* shearing box: fixed-point sweeps per step (0 = 8, at most 64);
                                with maxwell_tol > 0 the most sweeps a step may take */
    double maxwell_tol;      /* shearing box: 0 = always maxwell_iters sweeps; > 0 = stop after
                                the first sweep k with max|F^{k+1} - F^k| <= maxwell_tol *
                                max|F^{k+1}| over the six interior field components (FP32
                                comparison, decided on the device; Sec. 2.2 leaves the
                                stopping rule open) */
    uint32_t flags;          /* PIC_BOX_* */
    void* stream;            /* hipStream_t */
} pic_box_desc;

typedef struct pic_box pic_box;
typedef struct pic_batch pic_batch;

/* Sizes of the caller-owned memory of a box (pic_box_layout).  Field and current arrays are
   guarded: a component array holds pitch_z * field_planes floats, the interior point (i,j,k)
   at (32 + i) + pitch_y (2 + j) + pitch_z (2 + k) (k term 0 in 2D: no z guards), with
   pitch_y >= field_pitch_min[0] and pitch_z >= pitch_y * (n[1] + 4), both multiples of 32 (the
   interior x = 0 of every row starts a 128-byte line).  Particle arrays are dense, one
   element per slot. */
typedef struct pic_box_layout_info {
    int64_t workspace_bytes;    /* the workspace block (sort buffers, tile offsets, counters,
                                   reductions, reinjection table, the unfused record with
                                   PIC_BOX_UNFUSED) */
    int32_t field_sets;         /* field sets: 3 for the shearing box (F^n and the fixed-point
                                   iterates of Sec. 2.2), 1 otherwise */
    int32_t current_arrays;     /* current arrays per component: 2 for the shearing box (the
                                   J' transport of Sec. 2.2 writes the second), 1 otherwise */
    int32_t field_pitch_min[2]; /* smallest pitch_y, pitch_z (elements) */
    int32_t field_rows;         /* (n[1] + 4) * field_planes */
    int32_t field_planes;       /* n[2] + 4 in 3D, 1 in 2D */
    int64_t field_elems_min;    /* floats per field or current array at the smallest pitches */
    int64_t particle_elems[2];  /* elements per particle array of each species: capacity + 1 */
    int32_t has_id;             /* the id arrays are needed (ids carried) */
    int32_t has_dr;             /* the displacement arrays are needed (displacement escape) */
} pic_box_layout_info;

/* Caller-owned device memory of a box (pic_box_create).  Every pointer is device memory,
   256-byte aligned, and must outlive the box; the library reads and writes it on the box
   stream only.  Unused entries (sets beyond field_sets, the second current array outside the
   shearing box, species beyond n_species, off[..][..][2] in 2D, id and dr where the layout does
   not need them) are ignored. */
typedef struct pic_box_mem {
    float* field[3][6];          /* field set s: Bx By Bz Ex Ey Ez (the frame's evolved
                                    variables); pic_box_info.field_set names the set holding the
                                    fields after each step */
    float* current[2][3];        /* Jx Jy Jz; pic_box_info.current_array names the one holding the
                                    current of the last step */
    int32_t field_pitch[2];      /* pitch_y, pitch_z of every field and current array (0, 0: the
                                    smallest) */
    int32_t* cell[2][2];         /* [species][copy]: the two copies alternate between pushes */
    float* off[2][2][3];         /* [species][copy][axis], axis < dim */
    float* u[2][2][3];
    uint32_t* id[2][2];
    float* dr[2][2][3];
    void* workspace;             /* pic_box_layout_info.workspace_bytes or more */
    int64_t workspace_bytes;
} pic_box_mem;

/* The sizes a box of this descriptor needs on caller memory.  Host only (no device call).
   PIC_EINVAL for a descriptor pic_box_create would reject. */
int32_t pic_box_layout(const pic_box_desc* desc, pic_box_layout_info* out);
/* The workspace part of pic_box_layout. */
int32_t pic_workspace_bytes(const pic_box_desc* desc, int64_t* bytes);
/* Device and pinned host bytes the library currently holds: library-owned boxes, their
   unfused records and the batched-step staging of pic_step.  Boxes on caller memory and
   pic_batch objects add nothing. */
int32_t pic_allocated_bytes(int64_t* device_bytes, int64_t* host_bytes);

typedef struct pic_box_info {
    int64_t step;            /* steps taken */
    double t;                /* t^n = step*dt */
    double dys;              /* shearing box: Delta y_s(t) reduced mod n[1] (Sec. 2.1) */
    double a;                /* expanding box: l(t) of the expanding axes */
    int64_t n_particles[2];  /* particles in each species' arrays: those that escaped in the
                                last step (probabilistic escape) still hold a slot, with cell
                                -1, until the next sort drops them */
    uint32_t errors;         /* sticky PIC_DERR_* bits */
    int64_t n_slow;          /* particles handled outside their tile (counter) */
    int64_t n_escaped;       /* probabilistic escapes (counter) */
    /* FP64 reductions: sum E_c^2/8pi, sum B_c^2/8pi (c = x,y,z), kinetic energy
       sum m(gamma-1), momentum sum m u (particle sums skip the escaped particles) */
    double field_energy_E[3], field_energy_B[3];
    double kinetic_energy;
    double momentum[3];
    int64_t n_sort_migrations; /* sorts done by the neighbour-migration counting sort */
    int64_t n_sort_fallbacks;  /* of those, sorts that found a particle beyond the
                                  neighbouring tiles and fell back to the radix sort */
    int32_t maxwell_sweeps;    /* shearing box: fixed-point sweeps of the last Maxwell step
                                  (0 before the first step and for the other frames) */
    double pressure[3];        /* sum m u_c^2 / gamma (c = x,y,z): the diagonal of the kinetic
                                  stress; over the box volume, (sum of the three)/3 is the
                                  pressure n k T of the plasma-beta diagnostic of Sec. 4.2 */
    int64_t n_superluminal;    /* shearing box with PIC_BOX_COUNT_SUPERLUMINAL (counter, else
                                  0): particle pushes whose effective
                                  velocity u'/gamma' + v_s, v_s at the midpoint x of the move,
                                  exceeded c (eq. OAx; Sec. 2.1 leaves the correction to other
                                  work: counted, not corrected) */
    int32_t field_set;         /* the field set (pic_box_mem.field[s]) holding the fields */
    int32_t current_array;     /* the current array (pic_box_mem.current[a]) holding the current
                                  of the last step */
    int32_t particle_copy[2];  /* per species, the particle copy (pic_box_mem.cell[s][k], ...)
                                  holding the particles, in slot order */
} pic_box_info;

/* Create a box (the state of Secs. 2.1, 3.1, 4.1: fields on the Yee grid, particles of up to
   two species).  mem != NULL: the box lives in the caller's buffers (pic_box_mem, sized by
   pic_box_layout) and the library never allocates device or host memory for it; PIC_EINVAL
   for a missing or misaligned buffer or a bad pitch, PIC_ENOMEM for a workspace below
   pic_workspace_bytes.  mem == NULL: the library allocates the same buffers in one device
   allocation (PIC_ENOMEM if it fails).  Validates the descriptor (PIC_EINVAL: unsupported
   combination, CFL, capacity).  Fields and currents start at zero (cleared on the box stream)
   and the box holds no particles.  *out is set only on success. */
int32_t pic_box_create(const pic_box_desc* desc, const pic_box_mem* mem, pic_box** out);

/* Free the box and the memory the library allocated for it (synchronises the box stream);
   caller-owned buffers are untouched.  NULL is accepted. */
int32_t pic_box_destroy(pic_box* box);

/* Copy fields in or out: E_dev/B_dev/J_dev hold 3 component arrays of n0*n1*n2 floats.
   pic_set_fields also fills the guard cells at the current time. */
int32_t pic_set_fields(pic_box* box, const float* E_dev, const float* B_dev);
int32_t pic_get_fields(pic_box* box, float* E_dev, float* B_dev);
/* the current of the last step (J' for the shearing box, l J' for the expanding box, Sec. 3.1),
   after the guard fold and (shearing box) the J' transport of Sec. 2.2 */
int32_t pic_get_current(pic_box* box, float* J_dev);

/* Load n particles of one species (layout above; id_dev NULL -> ids 0..n-1, dr_dev NULL -> 0);
   the next pic_tile_sort (or pic_step) sorts them.  Asynchronous on the box stream: the input
   buffers must stay valid until the stream has passed this call.  PIC_ECAP if n exceeds the
   capacity, PIC_EINVAL on a bad species. */
int32_t pic_set_particles(pic_box* box, int32_t species, int64_t n, const int32_t* cell_dev,
                          const float* off_dev, const float* u_dev, const uint32_t* id_dev,
                          const float* dr_dev);
/* Copy the live particles of one species out in the box's current order (synchronises).
   *n_out receives the count; the arrays must hold pic_box_info.n_particles values.
   Any output pointer may be NULL. */
int32_t pic_get_particles(pic_box* box, int32_t species, int64_t* n_out, int32_t* cell_dev,
                          float* off_dev, float* u_dev, uint32_t* id_dev, float* dr_dev);
/* The permutation of the last tile sort: perm_dev[i] = index, in the order before that sort,
   of the particle in sorted position i (live particles only); offsets_dev receives the
   n_tiles+1 tile offsets.  Synchronises. */
int32_t pic_get_sort(pic_box* box, int32_t species, int32_t* perm_dev, int32_t* offsets_dev,
                     int32_t* n_tiles_out);

/* The record of the last pic_gather_push made without PIC_FUSE_DEPOSIT: per particle, in the
   slot order pic_get_particles returns after that push, the old cell (linear index, as at the
   boundary), the old in-cell offsets (off_dev: dim arrays of n) and the FP32 displacement of
   the deposit (disp_dev: 3 arrays of n; comoving x' - x^n in the shearing box, Sec. 2.2;
   primed in the expanding box, Sec. 3.2).  The new position is the old one moved by this
   displacement (plus, in the shearing box, the shear move of Sec. 2.2) under the FP32
   renormalisation and the boundary conditions (Sec. 2.1): the record lets a caller check that
   integer layer bit for bit.  *n_out receives the count; any output pointer may be NULL.
   PIC_ESTATE if the last push was fused (or none was made since the particles were loaded).
   Synchronises. */
int32_t pic_get_push_record(pic_box* box, int32_t species, int64_t* n_out, int32_t* cell_dev,
                            float* off_dev, float* disp_dev);

/* Tile-shape autotuner.  For every supported tile shape (PIC_TUNE_BATCHED: those of the batched
   step) it re-tiles the box, sorts its particles (radix sort) and times the fused
   gather-push-deposit kernel with HIP events on the box stream, trials + 1 times (the first
   is a warm-up; the fastest of the rest counts).  The kernel writes into the spare particle
   buffers and the current array, so the box's particles, fields and time are unchanged; the
   current array holds no result until the next step, and error bits and counters are
   restored.  The box keeps the fastest shape among those that admit the neighbour-migration
   sort (any shape if none does), and its next sort is a radix sort.  tile_out[3] receives
   the shape; ms_out[i] (i < max_out, may be NULL) the time of candidate i in the order of
   the supported list; *n_out (may be NULL) the number of candidates.  Synchronises.
   PIC_ESTATE with no particles loaded or an unfused push awaiting pic_deposit; PIC_EINVAL for
   trials outside 1..64.  Tile-indexed workspace is sized at pic_box_create for every shape. */
int32_t pic_autotune(pic_box* box, uint32_t flags, int32_t trials, int32_t* tile_out,
                     float* ms_out, int32_t max_out, int32_t* n_out);

/* The supported tile shapes of a dimension (PIC_TUNE_BATCHED: those of the batched step), in
   the order pic_autotune reports them, the default first: shapes_out[3*i + k] (host memory,
   room for max_out shapes) receives edge k of shape i.  Returns the number of shapes (it may
   exceed max_out), or PIC_EINVAL for a dimension other than 2 or 3. */
int32_t pic_tile_candidates(int32_t dim, uint32_t flags, int32_t* shapes_out, int32_t max_out);

/* ---- the hot path (each call acts on nb boxes; nb = 1 is the single-box case) ---- */

/* Tile counting sort (stable): key = tile of the particle's cell, dead particles go to a
   dead bin and are dropped.  Produces the permutation used by the next pic_gather_push and
   the per-tile offsets.  After a push the particles are still grouped by the tiles of the
   previous sort and each moved less than a cell, so (on tile grids with whole tiles and one
   or at least three tiles per axis) the sort only counts moves to the neighbouring tiles;
   a particle found farther away sends that sort to the general radix sort on the device.
   Both give the same permutation.  PIC_ESTATE while an unfused push awaits pic_deposit. */
int32_t pic_tile_sort(pic_box* const* boxes, int32_t nb, uint32_t flags);

/* Field gather at x^n, push u^{n-1/2} -> u^{n+1/2} with the frame's pusher (Boris;
   the shearing-box operator of Sec. 2.2, eq. OAu_disc; the expanding-box operator of
   Sec. 3.2, eq. EBu_disc), position update (Secs. 2.2, 3.2) with the boundary conditions
   (shearing-periodic x, Sec. 2.1), leaky-box displacement and escape test (Sec. 4.1 or the
   probabilistic rule).  With PIC_FUSE_DEPOSIT it also deposits the charge-conserving
   current (Esirkepov) into the box current; without it the old positions are kept for
   pic_deposit.  Requires a pic_tile_sort since the last push. */
int32_t pic_gather_push(pic_box* const* boxes, int32_t nb, uint32_t flags);

/* Charge-conserving current of the last unfused pic_gather_push (PIC_ESTATE otherwise). */
int32_t pic_deposit(pic_box* const* boxes, int32_t nb, uint32_t flags);

/* PIC_REMAP_CURRENT: fold the current guard cells (periodic, or shearing-periodic with
   Delta y_s(t^{n+1/2})) after the J' transport of Sec. 2.2 along y by v_{s,y} dt/2.
   PIC_REMAP_FIELDS: fill the field guard cells at the current time.  Plain periodic
   folding/filling for non-shear frames. */
int32_t pic_shear_remap(pic_box* const* boxes, int32_t nb, uint32_t what);

/* One Maxwell step of the box frame: Yee leapfrog (plain, leaky), Yee with the scale
   factors of Sec. 3.2 (expanding), implicit midpoint with upwinded advection solved by
   fixed-point iteration (shearing box, Sec. 2.2): maxwell_iters sweeps, or with maxwell_tol
   > 0 sweeps until the tolerance is met, where each sweep reduces its largest change and
   largest value on the device and the sweeps after the first converged one return at once
   (no host round trip; PIC_DERR_NOCONVERGE latches if none converges).  Advances the box
   time by dt. */
int32_t pic_maxwell_step(pic_box* const* boxes, int32_t nb, uint32_t flags);

/* Escape compaction: the tile sort with the dead bin, which removes the particles marked
   by the probabilistic escape, and the survivor count (read with pic_box_get). */
int32_t pic_escape_compact(pic_box* const* boxes, int32_t nb, uint32_t flags);

/* One whole step: sort, fused gather-push-deposit, current fold, Maxwell, field guards.
   Without flags the boxes are stepped one after another.  With PIC_STEP_BATCHED every stage
   runs as one launch per kernel over all nb boxes (independent boxes of any frame and size,
   sharing one stream; 2D tiles 16x16 or 8x8, 3D 8x8x8): per-box argument tables are staged in
   pinned host memory, copied once per step, and each launch maps its workgroups to boxes
   through a prefix table.  The sorts of a batched step use the neighbour-migration counting
   sort only; a particle found beyond the neighbouring tiles latches PIC_DERR_SORT on its box
   (that box's sort is then not valid).  Results equal the unbatched step's up to the order of
   the FP32 additions of the tile-halo current.  PIC_EINVAL if the boxes do not share one
   stream, appear twice or have an unsupported tile shape.
   With PIC_STEP_GRAPH the table transfer and the launches of the batched step are captured
   once as a HIP graph (stream capture on the shared stream, which must not be the null
   stream) and replayed on later steps of the same box set with the same launch shapes: the
   graph's copy node reads the tables the host has just written, so every replay runs that
   step's arguments.  The first box holds up to 8 graphs (least recently used evicted); they are
   freed with it.  Results are identical to the batched step without graphs.  The first box
   stages the tables in memory the library allocates for it, so it must be a library-owned box
   (PIC_EINVAL for a box on caller memory: step those with pic_step_batch). */
int32_t pic_step(pic_box* const* boxes, int32_t nb, uint32_t flags);

/* A batched step's staging on caller-owned memory: dev (device) and host (pinned host, e.g. a
   torch pin_memory tensor) of `bytes` each, 256-byte aligned; each holds two halves that
   alternate between steps, so one step's argument tables may take up to bytes/2
   (pic_step_table_bytes).  `stream` (a hipStream_t) is the stream of the boxes it steps.  The
   batch also keeps the HIP graphs of PIC_STEP_GRAPH (freed with it).  It allocates no memory.
   PIC_EINVAL for NULL or misaligned pointers or bytes below 2 x 4096. */
int32_t pic_batch_create(void* dev, void* host, int64_t bytes, void* stream, pic_batch** out);
int32_t pic_batch_destroy(pic_batch* batch); /* synchronises the stream; NULL accepted */
/* pic_step with PIC_STEP_BATCHED (flags may add PIC_STEP_GRAPH) whose argument tables are
   staged in the batch's buffers: the batched step for boxes on caller memory.  PIC_ENOMEM (and
   nothing stepped) if the tables exceed half the staging; PIC_EINVAL if the boxes do not use
   the batch's stream. */
int32_t pic_step_batch(pic_batch* batch, pic_box* const* boxes, int32_t nb, uint32_t flags);
/* Bytes of argument tables the next batched step of these boxes takes (host only: nothing is
   queued and the boxes are unchanged). */
int32_t pic_step_table_bytes(pic_box* const* boxes, int32_t nb, int64_t* bytes);

/* Synchronise the box stream and report time, counts, errors and (FP64) reductions. */
int32_t pic_box_get(pic_box* box, pic_box_info* info);

/* Resume from a checkpoint: set the step counter n of the box (t^n = n dt), on which the
   shearing offset Delta y_s(t) (Sec. 2.1), the scale factor l(t) (Sec. 3.1) and the Philox
   counters of the escape rules (id, step) depend, and refill the field guard cells at t^n.  A
   checkpoint is the fields (pic_get_fields), the particles with ids and displacements
   (pic_get_particles; those with cell -1 have escaped and are left out) and n; a box created
   from the same descriptor and loaded with them (pic_set_fields, pic_set_particles, then
   pic_set_step) continues the run with the same random stream.  Counters restart at zero.
   PIC_EINVAL for n < 0; PIC_ESTATE while an unfused push awaits pic_deposit. */
int32_t pic_set_step(pic_box* box, int64_t step);

#define PIC_HIST_MAX_BINS 4096

/* Particle energy distribution of one species (the diagnostic of Sec. 4.2): the kinetic
   energy of each particle that has not escaped, gamma - 1 = u.u / (1 + sqrt(1 + u.u)) in FP64 from its FP32
   momentum (units of m c^2), is placed by the nbins + 1 edges (host memory, FP64, strictly
   increasing and finite): counts_out[0] receives the particles below edges[0], counts_out[1 + b]
   those in [edges[b], edges[b + 1]), counts_out[nbins + 1] those at or above edges[nbins]
   (and any non-finite energy: the momentum latches PIC_DERR_NAN first).  counts_out: nbins + 2
   uint64 in host memory.  Synchronises.  PIC_EINVAL for nbins outside 1..PIC_HIST_MAX_BINS,
   edges not increasing, a bad species or NULL pointers. */
int32_t pic_energy_histogram(pic_box* box, int32_t species, const double* edges, int32_t nbins,
                             uint64_t* counts_out);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
   loops, harnesses that forbid hipMalloc): pic_energy_histogram with the same arguments,
   results and errors, whose scratch (the device copy of the edges and the counts being summed)
   is one static device array per GPU instead of the box's buffers.  It calls no hipMalloc,
   hipFree or other allocating routine.  The array holds PIC_HIST_STATIC_MAX_BINS bins (about
   64 KiB); nbins above it is PIC_EINVAL.  The box's device must be the current device.  Every
   call on one GPU shares that GPU's array, which keeps the last call's contents (the counts are
   cleared by a kernel at the start of each call): calls that overlap on one GPU, from several
   host threads or on several streams, race.  Synchronises. */
#define PIC_HIST_STATIC_MAX_BINS 4096
int32_t pic_energy_histogram_static(pic_box* box, int32_t species, const double* edges,
                                    int32_t nbins, uint64_t* counts_out);

/* Measurement utility, not part of the method: a plain streaming device-to-device copy of
   nbytes (a multiple of 16; both pointers 16-byte aligned device memory owned by the caller)
   on `stream` (a hipStream_t, NULL for the default stream), asynchronous.  Its known traffic
   (nbytes read, nbytes written) calibrates hardware memory counters.  PIC_EINVAL for a bad
   size or alignment. */
int32_t pic_device_copy(void* dst, const void* src, int64_t nbytes, void* stream);

/* Static description of a pic_status. */
const char* pic_status_str(int32_t status);

#ifdef __cplusplus
}
#endif
#endif
