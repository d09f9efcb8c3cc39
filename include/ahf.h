/*
 * ahf.h -- C ABI of the MI355X adaptive density hierarchy library (libahf.so).
 *
 * The library builds the grid hierarchy of AHF (Knollmann & Knebe, "AHF:
 * AMIGA's Halo Finder", Sect. 2.1): a domain grid covering the periodic box,
 * particle-density assignment with triangular-shaped-cloud (TSC) weights,
 * refinement of every cell whose particle count exceeds the threshold into
 * 8 half-size cells, repeated until no cell needs refinement, and the grid
 * tree of isolated refinements linked to the coarser volume that holds them.
 *
 * Conventions shared by every entry point
 *  - Positions: a particle at unit-box coordinate x is given as X + f quanta
 *    of 2^-21 per axis, X a uint32 below 2^21 and f a float in [0, 1).
 *  - Levels: level 0 is the domain grid with 2^g cells per axis; level L has
 *    b = g + L bits per axis.  Cell (x, y, z) of level L has the Morton key
 *    with bit 3j+2 = x_j, bit 3j+1 = y_j, bit 3j = z_j (j < b).
 *  - S_L: the cells of level L (level 0: all 2^{3g}; level L >= 1: the 8
 *    children of every refined cell of level L-1, empty children included).
 *    A cell is refined when its particle count is strictly greater than the
 *    threshold (dom_ref on level 0, ref_ref above), below the level cap.
 *  - The mass field of level L holds, for every particle inside S_L, its TSC
 *    share on the cells within one cell of it (periodic).  It is stored as
 *    bricks of 2x2x2 cells; each brick is keyed by its parent cell of level
 *    L-1 and the bricks cover every cell within one cell of S_L.  Cells of a
 *    brick that lie farther from S_L hold 0.  Level 0 has every brick.
 *  - Device pointers are HIP device addresses; host pointers are marked.
 *  - Every call returns an ahf_status; on failure *out parameters are set to
 *    NULL/0 and ahf_last_error() describes the failure.  No call throws.
 *  - Calls on one context are not thread-safe; use one context per thread.
 */
#ifndef AHF_H
#define AHF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ahf_status;
enum {
    AHF_OK = 0,
    AHF_PENDING = 1,       /* ahf_poll only: the request has not finished  */
    AHF_EINVAL = -1,       /* bad argument or out-of-range particle coordinate */
    AHF_ENOMEM = -2,       /* device or host allocation failed              */
    AHF_EDEVICE = -3,      /* a HIP runtime call failed                     */
    AHF_ELIMIT = -4,       /* size beyond what the library or budget allows  */
    AHF_EBUSY = -5,        /* server queue full                             */
    AHF_ENOTFOUND = -6,    /* unknown ticket                                */
    AHF_ECANCELED = -7     /* request released before it finished           */
};

/* flags of ahf_params */
#define AHF_NO_LABELS 1u   /* ahf_build_hierarchy skips the grid tree        */
#define AHF_SUBSTRUCTURE 2u /* ... and classifies it into host structures and
                                substructures (needs the grid tree)          */
#define AHF_DENSITY_CRITERION 4u /* refine where a cell's TSC particle density
                                (its deposited mass / mass_scalar, particles
                                per cell) exceeds the threshold, as the paper
                                states the criterion (Sect. 2.1), instead of
                                its particle count; needs equal masses
                                (mass NULL, mass_scalar > 0).  Flags then
                                rest on FP32 sums: a cell within ~1e-5 of the
                                threshold may decide differently from an
                                exact computation                            */

typedef struct ahf_ctx ahf_ctx;
typedef struct ahf_hierarchy ahf_hierarchy;
typedef struct ahf_server ahf_server;

/* Device memory callbacks.  alloc returns a device pointer of at least
 * `bytes` usable in stream order on `stream`, or NULL; free releases it. */
typedef void *(*ahf_alloc_fn)(void *user, size_t bytes, void *stream);
typedef void (*ahf_free_fn)(void *user, void *ptr, size_t bytes, void *stream);

typedef struct {
    uint32_t struct_size;  /* sizeof(ahf_ctx_desc) */
    int32_t device;        /* HIP device ordinal */
    ahf_alloc_fn alloc;    /* NULL: the library's own caching pool on hipMalloc */
    ahf_free_fn free;
    void *user;
} ahf_ctx_desc;

/* Parameters (Sect. 2.1 and 2.3 of the paper: DomGrid, DomRef, RefRef). */
typedef struct {
    uint32_t struct_size;    /* sizeof(ahf_params) */
    uint32_t dom_grid_log2;  /* g: DomGrid = 2^g cells per axis, 1..10      */
    double dom_ref;          /* level-0 threshold: refine if count > dom_ref */
    double ref_ref;          /* threshold on refined levels                  */
    uint32_t max_levels;     /* refinement levels beyond the domain grid;
                                g + max_levels <= 21                         */
    uint32_t connectivity;   /* 6, 18 or 26 (0 means 26): adjacency of the
                                isolated refinements                          */
    uint32_t flags;          /* AHF_NO_LABELS, AHF_SUBSTRUCTURE,
                                AHF_DENSITY_CRITERION                        */
} ahf_params;

/* Particle snapshot.  All arrays are device pointers of n elements, borrowed:
 * they must stay valid and unchanged until the build has passed on its stream
 * (or, for the server, until ahf_poll returns something other than PENDING).
 * fx/fy/fz may be NULL (offsets 0).  mass may be NULL (every particle weighs
 * mass_scalar). */
typedef struct {
    uint64_t n;              /* < 2^32 */
    const uint32_t *x, *y, *z;
    const float *fx, *fy, *fz;
    const float *mass;
    double mass_scalar;
} ahf_particles;

/* One level of a built hierarchy.  Device pointers stay valid until the
 * hierarchy is freed; NULL marks data that is not there (see each field). */
typedef struct {
    uint32_t level;
    uint32_t bits;                 /* b = g + level                              */
    uint64_t n_cells;              /* |S_L|                                      */
    uint64_t n_refined;            /* cells of S_L that are refined              */
    uint64_t n_particles;          /* particles inside S_L                       */
    uint64_t n_bricks;             /* bricks of the mass field                   */
    uint64_t n_patches;            /* isolated refinements (level >= 1, labelled) */
    const uint64_t *cell_key;      /* [n_cells] ascending; NULL on level 0, where
                                      cell i has key i                          */
    const uint32_t *cell_start;    /* [n_cells] first position in the particle
                                      order (ahf_hierarchy_order)               */
    const uint32_t *cell_count;    /* [n_cells]                                  */
    const uint8_t *cell_refined;   /* [n_cells] 1 if refined                     */
    const int32_t *cell_patch;     /* [n_cells] patch id; NULL on level 0 or
                                      before labelling                          */
    const uint64_t *brick_key;     /* [n_bricks] ascending parent keys (level
                                      L-1); NULL on level 0 (brick i has key i) */
    const int32_t *brick_cell;     /* [n_bricks] index in S_L of the brick's
                                      first cell, or -1 when the brick holds only
                                      ghost cells; NULL on level 0 (8 i)        */
    const float *brick_mass;       /* [8 n_bricks] TSC mass per cell; cell d of
                                      a brick has key 8*brick_key + d           */
    const int32_t *patch_parent;   /* [n_patches] patch id on level L-1, -1 on
                                      level 1 (the domain grid is the root)      */
    const uint32_t *patch_ncells;  /* [n_patches] cells of S_L in the patch      */
    const uint64_t *patch_nparticles; /* [n_patches]                            */
    const double *patch_mass;      /* [n_patches] particle mass in the patch     */
    double total_cell_mass;        /* sum of brick_mass (FP64 sum)               */
    double total_particle_mass;    /* mass of the particles inside S_L (FP64)    */
    const int32_t *patch_struct;   /* [n_patches] structure of each patch (see
                                      ahf_hierarchy_structures); NULL before
                                      classification                           */
} ahf_level_view;

/* Host structures and substructures of the grid tree (Sect. 2.1 of the
 * paper: the tree is walked from coarse to fine; where a patch splits, the
 * child with the most particles continues the parent's structure and the
 * others start substructures of it, recursively).  Every level-1 patch starts
 * a host structure; ties go to the lower patch id; structures are numbered by
 * (start level, start patch).  Device arrays of n_structures entries. */
typedef struct {
    uint64_t n_structures;
    const int32_t *host;   /* structure it branched off, -1 for a host       */
    const int32_t *level;  /* level of its first (coarsest) patch            */
    const int32_t *patch;  /* that patch's id on its level                   */
    const int32_t *depth;  /* 0 host, 1 substructure, 2 sub-substructure ... */
} ahf_structures;

const char *ahf_last_error(void);

ahf_status ahf_ctx_create(const ahf_ctx_desc *desc, ahf_ctx **out);
void ahf_ctx_destroy(ahf_ctx *ctx);

/*
 * Build the hierarchy of one snapshot on `stream` (a hipStream_t; NULL =
 * the default stream).  Steps: Morton keys and their stable sort; per
 * level, cell counts, refinement flags, TSC deposit, FP64 totals; the
 * grid tree unless AHF_NO_LABELS.  Returns when the hierarchy is complete
 * on the stream (the call synchronises the stream).  Errors: AHF_EINVAL for
 * bad parameters (checked before any launch) or a coordinate >= 2^21
 * (detected on the device), AHF_ENOMEM, AHF_EDEVICE.
 */
ahf_status ahf_build_hierarchy(ahf_ctx *ctx, const ahf_particles *particles,
                               const ahf_params *params, void *stream,
                               ahf_hierarchy **out);

/*
 * Grid tree of Sect. 2.1: on every level L >= 1 the connected components of
 * S_L (params.connectivity, periodic) are the isolated refinements.  Patch
 * ids follow the smallest Morton key of each component; a patch's parent is
 * the patch of level L-1 containing its parent cells.  Fills cell_patch and
 * the patch arrays of every level view.  Idempotent.
 */
ahf_status ahf_label_refinements(ahf_ctx *ctx, ahf_hierarchy *h, void *stream);

ahf_status ahf_hierarchy_num_levels(const ahf_hierarchy *h, uint32_t *out);
ahf_status ahf_level_get(const ahf_hierarchy *h, uint32_t level, ahf_level_view *out);

/* Classifies a labelled hierarchy into host structures and substructures
 * (done by ahf_build_hierarchy when params.flags has AHF_SUBSTRUCTURE).
 * Returns when it is complete.  AHF_EINVAL if the hierarchy is unlabelled. */
ahf_status ahf_classify_substructure(ahf_ctx *ctx, ahf_hierarchy *h, void *stream);

/* The structures of a classified hierarchy (AHF_EINVAL before). */
ahf_status ahf_hierarchy_structures(const ahf_hierarchy *h, ahf_structures *out);

/* Particle order: sorted_idx[i] is the input index of the i-th particle in
 * ascending B-bit Morton key (B = g + max_levels), ties by input index.  The
 * particles of every cell of every level are contiguous in this order. */
ahf_status ahf_hierarchy_order(const ahf_hierarchy *h, const uint32_t **sorted_idx);

/*
 * Builds sized ahead.  After a build, the context remembers, per parameter
 * set and size class (half octaves of n), how many cells each level refined
 * and how many bricks the next level got, per particle.  A later build of
 * that class is then enqueued level after level without the host waiting
 * for any level's counts: every level is sized from the remembered counts
 * (plus 15% and 64), the kernels read the true counts on the device, and a
 * level that outgrows its room is detected on the device; that build is then
 * redone with one host wait per level, which also updates the plan.  The
 * results are the same either way.  Planning is off by default: a single
 * build runs slightly faster with its per-level waits (they are hidden behind
 * the running deposits, and without them the next levels' cell kernels share
 * the GPU with the deposits, which are the longer chain).  It is what lets a
 * build run with no host involvement at all (ahf_batch_create records planned
 * builds into a graph).  Disabling it also forgets the plans.  (Not used with
 * AHF_DENSITY_CRITERION.)
 */
ahf_status ahf_ctx_set_planning(ahf_ctx *ctx, int enable);

typedef struct {
    uint32_t struct_size;   /* sizeof(ahf_build_info) */
    uint32_t planned;       /* 1: the levels were sized ahead                */
    uint32_t replanned;     /* 1: a planned attempt outgrew its room first    */
    uint32_t host_waits;    /* host waits for level counts during the build   */
    uint64_t device_bytes;  /* device memory the hierarchy holds              */
    uint32_t sort_key_bits; /* key bits the radix sort ordered by (3 B less the
                             * low bits it left out)                         */
    uint32_t sort_passes;   /* its 8-bit passes                               */
} ahf_build_info;
ahf_status ahf_hierarchy_build_info(const ahf_hierarchy *h, ahf_build_info *out);

/* Per-build stage times in milliseconds, for profiling: [0] keys + sort +
 * gather and [1] levels (device time between events on the build stream),
 * [2] labels and [3] total (host clock around the call).  n <= 4. */
ahf_status ahf_hierarchy_timings(const ahf_hierarchy *h, double *ms, uint32_t n);

void ahf_hierarchy_free(ahf_hierarchy *h);

/*
 * Tuning of the TSC deposit by build size.  A cell holding more than `heavy`
 * particles is summed by whole wavefronts in chunks instead of by one thread
 * (one threshold for level 0, one for level 1, one for the deeper levels);
 * batch_level1 records (2 or 4) are in flight per thread on level 1.  The
 * results do not depend on the tuning beyond FP32 summation order (every
 * choice is deterministic).  Defaults: heavy 64, 64, 64; batch 2.
 */
typedef struct {
    uint32_t struct_size;       /* sizeof(ahf_tuning) */
    uint32_t heavy_level0;      /* 1..64 */
    uint32_t heavy_level1;      /* 1..64 */
    uint32_t heavy_deeper;      /* 1..64 */
    uint32_t batch_level1;      /* 2 or 4 */
    int32_t sort_skip_digits;   /* -1: chosen by depth (2 when the keys hold 12 or more
                                 * levels below the domain grid, 1 for 9 or more, else 0);
                                 * else 0..2 low 8-bit key digits the radix sort leaves
                                 * out (never a bit of the domain grid); the particles
                                 * that only those digits order are then put in full-key
                                 * order, so the result is the same full stable sort */
} ahf_tuning;

/* Sets the context's tuning table: a build of n particles uses entries[i]
 * for the largest min_n[i] <= n (the defaults when there is none).  Host
 * arrays of n_entries (0 clears the table); copied.  AHF_EINVAL for values
 * out of range.  A server's workers take the table of the context the
 * server is created with. */
ahf_status ahf_ctx_set_tuning(ahf_ctx *ctx, uint32_t n_entries, const uint64_t *min_n,
                              const ahf_tuning *entries);
/* The tuning a build of n particles would use. */
ahf_status ahf_ctx_get_tuning(const ahf_ctx *ctx, uint64_t n, ahf_tuning *out);

/*
 * Kernel timing for profiling.  While enabled, the context records a pair of
 * HIP events around every launch of its main kernels, on the stream the
 * launch goes to ("keys", "rs_up", "rs_tscan", "rs_scatter", "gather",
 * "child_ranges", "heavy_chunk", "tile_deposit0", "tile_deposit1",
 * "tile_halo", "patches", "combine", "mark", "uf_hook", "uf_cross"; the three
 * "rs_" names are the tile histogram, tile offset and scatter kernels of each
 * radix-sort pass; "tile_deposit0/1" the dense tile deposits of levels 0 and
 * 1, "tile_halo" their halo adds, "patches" and "combine" the deposit of the
 * deeper levels).  Enabling or
 * disabling clears the accumulated times.  ahf_ctx_kernel_time returns the
 * number of launches and their summed device time (ms) for one name, reading
 * the events of finished builds.
 */
ahf_status ahf_ctx_set_profiling(ahf_ctx *ctx, int enable);
/* Restricts the timing to the listed kernel names (comma-separated, e.g.
 * "rs_scatter,gather"), so that the events cost nothing elsewhere; NULL or ""
 * times every name again.  Takes effect for launches made afterwards. */
ahf_status ahf_ctx_profile_only(ahf_ctx *ctx, const char *names);
ahf_status ahf_ctx_kernel_time(ahf_ctx *ctx, const char *kernel, uint64_t *launches,
                               double *total_ms);

/*
 * Label query on one hierarchy: patch id of each level-`level` cell given by
 * its Morton key (host arrays of n entries); -1 for a cell outside S_L and
 * for every cell of level 0 (the domain grid is the root of the tree).
 * The hierarchy must be labelled.  Synchronous on `stream`.
 */
ahf_status ahf_hierarchy_query_label(ahf_ctx *ctx, const ahf_hierarchy *h, uint32_t level,
                                     uint64_t n, const uint64_t *keys, int32_t *out,
                                     void *stream);

/*
 * The same label query for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the keys and results are staged in a static device array of
 * the library (3 MB, each GPU holding its own copy until the process ends)
 * instead of the context's workspace, and no device memory is allocated or
 * freed.  At most 262144 keys per call (AHF_ELIMIT beyond).  Every call on
 * one GPU shares that array: calls that overlap on one GPU race and must be
 * serialised by the caller.  Synchronous on `stream`; the hierarchy's device
 * must be the one it was built on.  Other errors as ahf_hierarchy_query_label.
 */
ahf_status ahf_hierarchy_query_label_static(const ahf_hierarchy *h, uint32_t level, uint64_t n,
                                            const uint64_t *keys, int32_t *out, void *stream);

/* ------------------------------------------------------------------ serving
 *
 * A server builds hierarchies of many snapshot sub-volumes concurrently:
 * n_streams worker threads, each with its own HIP stream and scratch space,
 * take admitted requests in submission order, so requests that arrive while
 * others are on the GPU start as soon as a worker and HBM are free and their
 * kernels overlap on the device.  A request is admitted when its estimated
 * footprint (inputs excluded) fits the HBM budget together with the device
 * memory the workers' contexts hold (finished results, cached blocks,
 * workspaces; for contexts with allocation callbacks, what they have
 * allocated and not freed) and the builds in flight.  To make room, cached
 * blocks are given back first, then finished results that no client holds
 * are evicted least recently used first, then idle workers' workspaces are
 * given back.  A result that ahf_poll or ahf_wait has handed out is held by
 * the client and never evicted until ahf_release.  If nothing runs and only
 * held results stand in the way, the waiting request fails with AHF_ELIMIT
 * rather than wait for ever.  Results do not depend on what else runs: every
 * build is deterministic.  All server calls are thread-safe; none may be in
 * progress when ahf_server_destroy is called.
 */
typedef struct {
    uint32_t struct_size;   /* sizeof(ahf_server_desc) */
    uint32_t n_streams;     /* concurrent builds, 1..16; with more than one,
                               each build keeps to its worker's one stream */
    uint32_t max_queue;     /* queued (not yet admitted) requests; 0 = 1024 */
    uint32_t flags;         /* reserved, 0 */
    uint64_t hbm_budget;    /* bytes for builds in flight + resident results;
                               0 = 80% of the free device memory at creation */
} ahf_server_desc;

typedef struct {
    uint64_t submitted, completed, failed, evicted, released;  /* released
                                  counts dropped results and canceled requests */
    uint64_t queued, running, resident;
    uint64_t bytes_in_use;     /* device memory of the workers' contexts + what
                                  the estimates of running builds add to it */
    uint64_t bytes_peak;       /* largest bytes_in_use seen at an admission or
                                  the end of a build */
    uint64_t bytes_results;    /* device memory of the resident results (part of
                                  bytes_in_use) */
} ahf_server_stats;

/* ctx supplies the device and the allocation callbacks; it must outlive the
 * server.  Errors: AHF_EINVAL, AHF_EDEVICE, AHF_ENOMEM. */
ahf_status ahf_server_create(ahf_ctx *ctx, const ahf_server_desc *desc, ahf_server **out);

/* Non-blocking.  The particle arrays are borrowed until ahf_poll/ahf_wait has
 * returned something other than AHF_PENDING for the ticket.  Errors:
 * AHF_EINVAL (parameters, as ahf_build_hierarchy), AHF_ELIMIT (the request
 * alone exceeds the budget), AHF_EBUSY (queue full). */
ahf_status ahf_submit(ahf_server *s, const ahf_particles *particles, const ahf_params *params,
                      uint64_t *ticket);

/* AHF_PENDING while queued or running; AHF_OK with *h borrowed from the
 * server: from then on the client holds the result, which stays valid (it is
 * never evicted) until ahf_release; the build's error status if it failed;
 * AHF_ECANCELED if it was released while still queued (the 4096 most recent
 * such tickets are remembered); AHF_ENOTFOUND for an unknown, released or
 * evicted ticket. */
ahf_status ahf_poll(ahf_server *s, uint64_t ticket, ahf_hierarchy **h);
/* as ahf_poll, but waits while the request is pending */
ahf_status ahf_wait(ahf_server *s, uint64_t ticket, ahf_hierarchy **h);

/* label query on a finished, resident request (see ahf_hierarchy_query_label) */
ahf_status ahf_query_label(ahf_server *s, uint64_t ticket, uint32_t level, uint64_t n,
                           const uint64_t *keys, int32_t *out);

/* Drops the result of a finished request (held or not), or cancels a queued
 * one (its poll then returns AHF_ECANCELED; releasing a canceled ticket again
 * forgets it).  A running request, or one with a label query in progress, is
 * released when that ends. */
ahf_status ahf_release(ahf_server *s, uint64_t ticket);

/* submit, admission, start and end times of a request in ms on the host's
 * steady clock (t[0..3]); start/end are 0 until they happen */
ahf_status ahf_ticket_times(ahf_server *s, uint64_t ticket, double *t);
ahf_status ahf_server_get_stats(ahf_server *s, ahf_server_stats *out);

/* Waits for running builds, frees every result. */
void ahf_server_destroy(ahf_server *s);

/* ------------------------------------------------------------------ halos
 *
 * Particle collection and iterative unbinding (Sect. 2.1, the paragraphs after
 * the classification of the grid tree; App. A).  Every structure of a
 * classified hierarchy is a prospective halo:
 * - its leaf is its patch on the deepest level its main branch reaches; its
 *   centre is the centre of mass of the leaf patch's particles (periodic
 *   minimum image relative to the lower corner of the leaf's smallest-key
 *   cell; a leaf without mass takes that cell's centre);
 * - a host collects the particles of its main-branch patch on the deepest
 *   level whose boundary contour, thr_{L-1} particles per level-(L-1) cell,
 *   lies below delta_vir times the background density (its start patch when
 *   none does); a substructure collects every particle within half the
 *   distance from its centre to its host's centre;
 * - the halo is then unbound in isolation: per round, the velocity of the halo
 *   is the mass-weighted mean of its particles' velocities; with the particles
 *   ordered by radius from the fixed centre (clamped below at half a position
 *   quantum; ties by index), r_vir is the radius of the last particle whose
 *   enclosed mean density (itself included) is at least delta_vir times the
 *   background; the potential is phi(r) = -G (int_r^r_vir M(<r')/r'^2 dr' +
 *   M_vir / r_vir) within r_vir, -G M_vir / r beyond (App. A, the halo
 *   truncated at r_vir; the enclosed mass is constant between particles); a
 *   particle whose kinetic energy per mass relative to the halo exceeds |phi|
 *   is removed; rounds repeat until none is (at most max_iter);
 * - the halo's particles are those left within r_vir.  A halo that never
 *   reaches the overdensity, or does not converge, keeps none (r_vir = M_vir
 *   = 0).
 * Units are the caller's: positions in box lengths, the particle masses of
 * the build, velocities as given, G as given; the background density is the
 * total particle mass per box volume.
 */
typedef struct {
    uint32_t struct_size;   /* sizeof(ahf_halo_params) */
    double delta_vir;       /* virial overdensity (the paper's mass functions use 340) */
    double G;               /* gravitational constant in the caller's units */
    uint32_t max_iter;      /* at most this many unbinding rounds (>= 1) */
    uint32_t large_from;    /* structures with at least this many possible candidates are
                             * unbound by the whole GPU together, the others by one
                             * workgroup each (0: 32768); the results do not depend on it
                             * beyond FP64 summation order */
} ahf_halo_params;

typedef struct ahf_halos ahf_halos;

/* Finds the halos of h, which must be labelled and classified.  p holds the
 * particles the hierarchy was built from (same device arrays or copies; n as
 * built); vx, vy, vz are device arrays of n velocities.  Waits for the work
 * on stream.  The result owns its device memory (ctx's allocator) until
 * ahf_halos_free.  Scratch space comes from ctx's workspace (kept for later
 * calls): one 64-byte record per particle, and per-candidate arrays of some
 * tens of bytes per possible candidate. */
ahf_status ahf_find_halos(ahf_ctx *ctx, const ahf_hierarchy *h, const ahf_particles *p,
                          const float *vx, const float *vy, const float *vz,
                          const ahf_halo_params *prm, void *stream, ahf_halos **out);

/* Device views of the halos, one per structure (structure order).  Halo s's
 * candidates and its particles are stored from cand_offset[s] on: cand[...]
 * the candidates' particle indices in radius order from the centre, ties by
 * index (cand_count[s] of them); member[...] the halo's particles in the same
 * order (member_count[s]), the innermost of the last round. */
typedef struct {
    uint64_t n_halos;
    const uint64_t *leaf;           /* leaf level << 32 | leaf patch id */
    const double *centre;           /* [3 n] x, y, z in [0, 1) */
    const double *radius;           /* collection radius of a substructure, 0 for a host */
    const uint64_t *cand_offset;    /* [n + 1] */
    const uint32_t *cand_count;
    const uint32_t *cand;
    const uint32_t *member_count;
    const uint32_t *member;
    const double *r_vir;
    const double *m_vir;
    const double *vel;              /* [3 n] the halo's velocity (last round) */
    const uint32_t *iterations;     /* unbinding rounds taken */
} ahf_halos_view;
ahf_status ahf_halos_get(const ahf_halos *hs, ahf_halos_view *out);
void ahf_halos_free(ahf_halos *hs);

/* ------------------------------------------------------------------ batches
 *
 * Many independent sub-volumes built by one graph launch.  The paper analyses
 * independent chunks of a simulation separately (Sect. 2.2.3, and Sect. 5.3 on
 * splitting a large volume); a batch builds a fixed set of such sub-volumes
 * again and again (for instance each time their particles have moved) with
 * no host involvement inside the run.
 *
 * ahf_batch_create builds every sub-volume twice on ctx's device: the first
 * build learns its level sizes, the second runs exactly as every run will
 * (sized ahead with no host wait per level, labels within the build, a status
 * block copied on the device) and sizes the batch's memory.  A run enqueues
 * every build at once: n_chains independent chains (1..16; each with its own
 * streams and scratch memory), the sub-volumes dealt to the chains largest
 * first; the host waits once, at ahf_batch_wait.  On return the batch has not
 * run yet.
 *
 * flags: AHF_BATCH_GRAPH records the builds into one HIP graph, so that a run
 * is one graph launch.  That recording is switched off in this version
 * (AHF_EINVAL): the HIP runtime faulted while ending the recording of these
 * multi-stream builds.
 *
 * parts[i] and params[i] describe sub-volume i (n >= 1 sub-volumes, each with
 * at least one particle, equal masses: mass NULL, and none of the flags
 * AHF_DENSITY_CRITERION and AHF_SUBSTRUCTURE; AHF_EINVAL otherwise).  The
 * particle arrays are borrowed for the life of the batch: every run reads them
 * at the same addresses, so the caller may rewrite their contents (not their
 * sizes) between runs.  Device memory comes from ctx's allocator; ctx must
 * outlive the batch.  The call first waits for stream (on which the caller
 * may have produced the particle arrays); the batch has streams of its own.
 */
typedef struct ahf_batch ahf_batch;
#define AHF_BATCH_GRAPH 1u
ahf_status ahf_batch_create(ahf_ctx *ctx, uint32_t n, const ahf_particles *parts,
                            const ahf_params *params, uint32_t n_chains, uint32_t flags,
                            void *stream, ahf_batch **out);

/* Enqueues one run after the work already on stream: every sub-volume is
 * rebuilt from the current contents of its particle arrays, and stream waits
 * for the run.  The hierarchies of the previous run are invalid from here
 * until ahf_batch_wait. */
ahf_status ahf_batch_run(ahf_batch *b, void *stream);

/* Waits for the run and completes the hierarchies from the status blocks the
 * run left on the device.  AHF_OK when every sub-volume built; else the first
 * failing sub-volume's error: AHF_ELIMIT when its particles now need more
 * cells or bricks on some level than the recorded sizes allow (create the
 * batch again), AHF_EINVAL for a coordinate >= 2^21, AHF_EDEVICE for a device
 * fault.  ahf_batch_status gives each sub-volume's status. */
ahf_status ahf_batch_wait(ahf_batch *b);
ahf_status ahf_batch_status(const ahf_batch *b, uint32_t i);

/* The hierarchy of sub-volume i after a successful wait, borrowed from the
 * batch (valid until the next run or ahf_batch_destroy; never freed by the
 * caller).  AHF_EINVAL before a run has completed or when sub-volume i failed. */
ahf_status ahf_batch_hierarchy(ahf_batch *b, uint32_t i, ahf_hierarchy **out);

/* Waits for a pending run and frees the graph, the hierarchies and the
 * chains' memory. */
void ahf_batch_destroy(ahf_batch *b);

#ifdef __cplusplus
}
#endif
#endif /* AHF_H */
