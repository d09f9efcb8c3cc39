/*
 * ahf_oracle.c -- plain, slow CPU oracle of the adaptive density hierarchy.
 *
 * TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the CPU-baseline
 * leg of the benchmark call it; the device library never links, imports or
 * calls anything here, and nothing here is shared with it.
 *
 * What it computes (Knollmann & Knebe, "AHF: AMIGA's Halo Finder",
 * Sect. 2.1, the paragraphs on the domain grid, the refinement criteria and the
 * grid tree), in double precision, with the readings below:
 *
 *  - The periodic unit box is covered by the domain grid of 2^g cells per
 *    axis (level 0).  A particle's position is X + f quanta of 2^-21, with X a
 *    21-bit integer and f in [0,1).  At level L the grid has b = g + L bits per
 *    axis and the particle's cell is X >> (21 - b) on each axis.
 *  - A cell is refined when the number of particles in it exceeds the
 *    threshold (DomRef on level 0, RefRef above); refinement stops at the
 *    level cap, at b = 21, or when no cell is refined.  A refined cell is
 *    covered by its 8 half-size children (all 8 exist, empty ones included).
 *    With the density criterion (Sect. 2.1 read literally: the particle
 *    density, from the TSC assignment, exceeds the threshold), the quantity
 *    compared is instead the TSC particle number of the cell, N_L(c) = sum
 *    over P_L of the particle's weight on c, in particles per cell.
 *  - S_L is the set of cells of level L, P_L the particles inside S_L.  The
 *    particles of P_L are assigned to the cells with triangular-shaped-cloud
 *    weights (Hockney & Eastwood): per axis, with u the in-cell offset in
 *    [0,1), cell i-1 gets (1-u)^2/2, cell i gets 3/4-(u-1/2)^2, cell i+1 gets
 *    u^2/2, all indices periodic.  The deposit targets are E_L, i.e. S_L plus every
 *    cell within one cell (Chebyshev) of S_L; cells of E_L outside S_L are
 *    "ghost" cells, never refined or labelled.  This keeps the mass of every
 *    level: sum over E_L of M equals the mass of P_L.
 *  - Grid tree: on every level L >= 1 the isolated refinements are the
 *    connected components of S_L (26-, 18- or 6-connectivity, periodic); a
 *    component is named by its smallest Morton key, patches are numbered in
 *    increasing order of that key, and a patch's parent is the patch of level
 *    L-1 holding the parent cells (level-1 patches hang off the domain grid,
 *    parent -1).
 *
 * Morton key of cell (x, y, z) at b bits: bit 3j+2 holds x_j, bit 3j+1 holds
 * y_j, bit 3j holds z_j.  The global particle order is the stable sort by the
 * key at B = g + max_levels bits (capped at 21), ties by input index.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_LEVELS 22

typedef struct {
    int b;
    uint64_t nS;
    uint64_t *S_key;
    uint32_t *S_count;
    uint32_t *S_start;
    uint8_t *S_flag;
    int32_t *S_patch;
    double *S_pmass;          /* mass of the particles in each cell */
    uint64_t nE;
    uint64_t *E_key;
    double *E_mass;
    double *E_num;   /* TSC particle number per cell of E_L (density criterion) */
    uint8_t *E_ghost;
    uint64_t nP;
    double tot_cell_mass;
    double tot_part_mass;
    uint64_t npatch;
    int32_t *patch_parent;
    uint64_t *patch_ncells;
    uint64_t *patch_npart;
    double *patch_mass;
} orc_level;

typedef struct {
    int nlev;
    int B;
    uint64_t n;
    uint32_t *order;
    orc_level lev[ORC_MAX_LEVELS];
} orc_hier;

/* ---------------------------------------------------------------- keys */

static uint64_t morton(uint32_t x, uint32_t y, uint32_t z, int bits)
{
    uint64_t k = 0;
    for (int j = 0; j < bits; j++) {
        k |= (uint64_t)((x >> j) & 1u) << (3 * j + 2);
        k |= (uint64_t)((y >> j) & 1u) << (3 * j + 1);
        k |= (uint64_t)((z >> j) & 1u) << (3 * j);
    }
    return k;
}

static void demorton(uint64_t k, int bits, uint32_t *x, uint32_t *y, uint32_t *z)
{
    uint32_t a = 0, b = 0, c = 0;
    for (int j = 0; j < bits; j++) {
        a |= (uint32_t)((k >> (3 * j + 2)) & 1u) << j;
        b |= (uint32_t)((k >> (3 * j + 1)) & 1u) << j;
        c |= (uint32_t)((k >> (3 * j)) & 1u) << j;
    }
    *x = a; *y = b; *z = c;
}

/* key of the cell displaced by (dx, dy, dz) cells, periodic at b bits */
static uint64_t neighbour(uint64_t k, int bits, int dx, int dy, int dz)
{
    uint32_t x, y, z;
    uint32_t mask = (bits >= 32) ? 0xffffffffu : ((1u << bits) - 1u);
    demorton(k, bits, &x, &y, &z);
    x = (uint32_t)((int64_t)x + dx) & mask;
    y = (uint32_t)((int64_t)y + dy) & mask;
    z = (uint32_t)((int64_t)z + dz) & mask;
    return morton(x, y, z, bits);
}

static int64_t find_key(const uint64_t *a, uint64_t n, uint64_t key)
{
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (a[mid] < key) lo = mid + 1; else hi = mid;
    }
    if (lo < n && a[lo] == key) return (int64_t)lo;
    return -1;
}

static uint64_t lower_bound(const uint64_t *a, uint64_t n, uint64_t key)
{
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (a[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

static int cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

typedef struct { uint64_t key; uint32_t idx; } keyidx;

static int cmp_keyidx(const void *a, const void *b)
{
    const keyidx *p = (const keyidx *)a, *q = (const keyidx *)b;
    if (p->key != q->key) return (p->key > q->key) - (p->key < q->key);
    return (p->idx > q->idx) - (p->idx < q->idx);
}

/* --------------------------------------------------------------- TSC */

/* TSC weight on the cell at offset a in {-1,0,1} for in-cell offset u */
static double tsc_weight(int a, double u)
{
    if (a < 0) return 0.5 * (1.0 - u) * (1.0 - u);
    if (a > 0) return 0.5 * u * u;
    return 0.75 - (u - 0.5) * (u - 0.5);
}

/* in-cell offset in [0,1) of coordinate (X, f) on a grid of b bits */
static double in_cell(uint32_t X, float f, int b)
{
    int k = 21 - b;
    uint32_t lo = X & ((1u << k) - 1u);
    return ((double)lo + (double)f) / (double)(1u << k);
}

static int in_connectivity(int dx, int dy, int dz, int conn)
{
    int s = abs(dx) + abs(dy) + abs(dz);
    if (s == 0) return 0;
    if (conn == 6) return s == 1;
    if (conn == 18) return s <= 2;
    return 1;
}

/* ------------------------------------------------------------ build */

static void free_level(orc_level *v)
{
    free(v->S_key); free(v->S_count); free(v->S_start); free(v->S_flag);
    free(v->S_patch); free(v->S_pmass);
    free(v->E_key); free(v->E_mass); free(v->E_num); free(v->E_ghost);
    free(v->patch_parent); free(v->patch_ncells); free(v->patch_npart); free(v->patch_mass);
    memset(v, 0, sizeof(*v));
}

void orc_free(orc_hier *h)
{
    if (!h) return;
    for (int L = 0; L < ORC_MAX_LEVELS; L++) free_level(&h->lev[L]);
    free(h->order);
    free(h);
}

/* components of S_L by breadth-first flood fill, numbered by smallest key */
static int label_level(orc_hier *h, int L, int conn)
{
    orc_level *v = &h->lev[L];
    uint64_t n = v->nS;
    v->S_patch = (int32_t *)malloc(sizeof(int32_t) * (n ? n : 1));
    uint64_t *queue = (uint64_t *)malloc(sizeof(uint64_t) * (n ? n : 1));
    if (!v->S_patch || !queue) { free(queue); return -1; }
    for (uint64_t i = 0; i < n; i++) v->S_patch[i] = -1;
    int32_t np = 0;
    for (uint64_t i = 0; i < n; i++) {
        if (v->S_patch[i] >= 0) continue;
        uint64_t head = 0, tail = 0;
        queue[tail++] = i;
        v->S_patch[i] = np;
        while (head < tail) {
            uint64_t c = queue[head++];
            for (int dx = -1; dx <= 1; dx++)
                for (int dy = -1; dy <= 1; dy++)
                    for (int dz = -1; dz <= 1; dz++) {
                        if (!in_connectivity(dx, dy, dz, conn)) continue;
                        uint64_t nk = neighbour(v->S_key[c], v->b, dx, dy, dz);
                        int64_t j = find_key(v->S_key, n, nk);
                        if (j >= 0 && v->S_patch[j] < 0) {
                            v->S_patch[j] = np;
                            queue[tail++] = (uint64_t)j;
                        }
                    }
        }
        np++;
    }
    free(queue);
    v->npatch = (uint64_t)np;
    uint64_t m = (uint64_t)(np ? np : 1);
    v->patch_parent = (int32_t *)malloc(sizeof(int32_t) * m);
    v->patch_ncells = (uint64_t *)calloc(m, sizeof(uint64_t));
    v->patch_npart = (uint64_t *)calloc(m, sizeof(uint64_t));
    v->patch_mass = (double *)calloc(m, sizeof(double));
    if (!v->patch_parent || !v->patch_ncells || !v->patch_npart || !v->patch_mass) return -1;
    for (int32_t p = 0; p < np; p++) v->patch_parent[p] = -1;
    for (uint64_t i = 0; i < n; i++) {
        int32_t p = v->S_patch[i];
        v->patch_ncells[p] += 1;
        v->patch_npart[p] += v->S_count[i];
        v->patch_mass[p] += v->S_pmass[i];
    }
    if (L >= 2) {
        orc_level *u = &h->lev[L - 1];
        /* cells are visited in increasing key order, so the first cell met of
           each patch is its smallest; its parent cell lies in S_{L-1}. */
        uint8_t *done = (uint8_t *)calloc(m, 1);
        if (!done) return -1;
        for (uint64_t i = 0; i < n; i++) {
            int32_t p = v->S_patch[i];
            if (done[p]) continue;
            done[p] = 1;
            int64_t j = find_key(u->S_key, u->nS, v->S_key[i] >> 3);
            v->patch_parent[p] = (j >= 0) ? u->S_patch[j] : -2;
        }
        free(done);
    }
    return 0;
}

/*
 * Build the hierarchy.  mass may be NULL (every particle then weighs
 * mass_scalar).  conn in {6, 18, 26}; labels=0 skips the grid tree.
 * Returns 0 on success, negative on bad arguments or memory exhaustion.
 */
int orc_build(uint64_t n, const uint32_t *X, const uint32_t *Y, const uint32_t *Z,
              const float *fx, const float *fy, const float *fz, const float *mass,
              double mass_scalar, int g, double dom_ref, double ref_ref, int max_levels,
              int conn, int labels, int density, orc_hier **out)
{
    *out = NULL;
    if (g < 1 || max_levels < 0 || g + max_levels > 21) return -1;
    if (conn != 6 && conn != 18 && conn != 26) return -1;
    if (isnan(dom_ref) || isnan(ref_ref)) return -1;
    if (n >= (1ull << 32)) return -1;
    for (uint64_t p = 0; p < n; p++)
        if (X[p] >= (1u << 21) || Y[p] >= (1u << 21) || Z[p] >= (1u << 21)) return -2;

    orc_hier *h = (orc_hier *)calloc(1, sizeof(orc_hier));
    if (!h) return -3;
    h->n = n;
    int B = g + max_levels;
    h->B = B;

    /* global order: stable sort by the B-bit key */
    keyidx *ki = (keyidx *)malloc(sizeof(keyidx) * (n ? n : 1));
    uint64_t *sorted = (uint64_t *)malloc(sizeof(uint64_t) * (n ? n : 1));
    h->order = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
    uint64_t *pcell = (uint64_t *)malloc(sizeof(uint64_t) * (n ? n : 1));
    int64_t *pidx = (int64_t *)malloc(sizeof(int64_t) * (n ? n : 1));
    if (!ki || !sorted || !h->order || !pcell || !pidx) goto oom;
    for (uint64_t p = 0; p < n; p++) {
        ki[p].key = morton(X[p] >> (21 - B), Y[p] >> (21 - B), Z[p] >> (21 - B), B);
        ki[p].idx = (uint32_t)p;
    }
    qsort(ki, n, sizeof(keyidx), cmp_keyidx);
    for (uint64_t p = 0; p < n; p++) { sorted[p] = ki[p].key; h->order[p] = ki[p].idx; }
    free(ki); ki = NULL;

    for (int L = 0; L <= max_levels; L++) {
        orc_level *v = &h->lev[L];
        int b = g + L;
        int shift = 21 - b;
        v->b = b;
        if (L == 0) {
            v->nS = 1ull << (3 * g);
            v->S_key = (uint64_t *)malloc(sizeof(uint64_t) * v->nS);
            if (!v->S_key) goto oom;
            for (uint64_t i = 0; i < v->nS; i++) v->S_key[i] = i;
        } /* else S_L was filled from F_{L-1} below */
        uint64_t nS = v->nS;
        v->S_count = (uint32_t *)calloc(nS ? nS : 1, sizeof(uint32_t));
        v->S_start = (uint32_t *)malloc(sizeof(uint32_t) * (nS ? nS : 1));
        v->S_flag = (uint8_t *)calloc(nS ? nS : 1, 1);
        v->S_pmass = (double *)calloc(nS ? nS : 1, sizeof(double));
        if (!v->S_count || !v->S_start || !v->S_flag || !v->S_pmass) goto oom;

        /* P_L and the per-cell counts */
        v->nP = 0;
        v->tot_part_mass = 0.0;
        for (uint64_t p = 0; p < n; p++) {
            pcell[p] = morton(X[p] >> shift, Y[p] >> shift, Z[p] >> shift, b);
            pidx[p] = find_key(v->S_key, nS, pcell[p]);
            if (pidx[p] >= 0) {
                double m = mass ? (double)mass[p] : mass_scalar;
                v->S_count[pidx[p]] += 1;
                v->S_pmass[pidx[p]] += m;
                v->nP += 1;
                v->tot_part_mass += m;
            }
        }
        /* start of each cell in the global order: particles whose level-L cell
           key is smaller */
        for (uint64_t i = 0; i < nS; i++)
            v->S_start[i] = (uint32_t)lower_bound(sorted, n, v->S_key[i] << (3 * (B - b)));

        /* E_L = S_L plus its one-cell ring */
        if (L == 0) {
            v->nE = nS;
            v->E_key = (uint64_t *)malloc(sizeof(uint64_t) * nS);
            if (!v->E_key) goto oom;
            memcpy(v->E_key, v->S_key, sizeof(uint64_t) * nS);
        } else {
            uint64_t *cand = (uint64_t *)malloc(sizeof(uint64_t) * (27 * nS + 1));
            if (!cand) goto oom;
            uint64_t nc = 0;
            for (uint64_t i = 0; i < nS; i++)
                for (int dx = -1; dx <= 1; dx++)
                    for (int dy = -1; dy <= 1; dy++)
                        for (int dz = -1; dz <= 1; dz++)
                            cand[nc++] = neighbour(v->S_key[i], b, dx, dy, dz);
            qsort(cand, nc, sizeof(uint64_t), cmp_u64);
            uint64_t ne = 0;
            for (uint64_t i = 0; i < nc; i++)
                if (i == 0 || cand[i] != cand[i - 1]) cand[ne++] = cand[i];
            v->nE = ne;
            v->E_key = (uint64_t *)realloc(cand, sizeof(uint64_t) * (ne ? ne : 1));
            if (!v->E_key) { free(cand); goto oom; }
        }
        v->E_mass = (double *)calloc(v->nE ? v->nE : 1, sizeof(double));
        v->E_num = (double *)calloc(v->nE ? v->nE : 1, sizeof(double));
        v->E_ghost = (uint8_t *)calloc(v->nE ? v->nE : 1, 1);
        if (!v->E_mass || !v->E_num || !v->E_ghost) goto oom;
        for (uint64_t e = 0; e < v->nE; e++)
            v->E_ghost[e] = find_key(v->S_key, nS, v->E_key[e]) < 0;

        /* TSC deposit of P_L onto E_L */
        for (uint64_t p = 0; p < n; p++) {
            if (pidx[p] < 0) continue;
            double m = mass ? (double)mass[p] : mass_scalar;
            double ux = in_cell(X[p], fx[p], b);
            double uy = in_cell(Y[p], fy[p], b);
            double uz = in_cell(Z[p], fz[p], b);
            for (int dx = -1; dx <= 1; dx++)
                for (int dy = -1; dy <= 1; dy++)
                    for (int dz = -1; dz <= 1; dz++) {
                        double w = tsc_weight(dx, ux) * tsc_weight(dy, uy) * tsc_weight(dz, uz);
                        uint64_t t = neighbour(pcell[p], b, dx, dy, dz);
                        int64_t e = find_key(v->E_key, v->nE, t);
                        if (e < 0) goto fail; /* cannot happen: t is within one cell of S_L */
                        v->E_mass[e] += m * w;
                        v->E_num[e] += w;
                    }
        }
        v->tot_cell_mass = 0.0;
        for (uint64_t e = 0; e < v->nE; e++) v->tot_cell_mass += v->E_mass[e];

        /* refinement */
        h->nlev = L + 1;
        if (L == max_levels || b >= 21) break;
        double thr = (L == 0) ? dom_ref : ref_ref;
        uint64_t nF = 0;
        for (uint64_t i = 0; i < nS; i++) {
            if (density) {
                /* the cell's TSC particle number: its entry in E_L */
                int64_t e = find_key(v->E_key, v->nE, v->S_key[i]);
                v->S_flag[i] = v->E_num[e] > thr;
            } else {
                v->S_flag[i] = (double)v->S_count[i] > thr;
            }
            nF += v->S_flag[i];
        }
        if (nF == 0) break;
        orc_level *w = &h->lev[L + 1];
        w->nS = 8 * nF;
        w->S_key = (uint64_t *)malloc(sizeof(uint64_t) * w->nS);
        if (!w->S_key) goto oom;
        uint64_t j = 0;
        for (uint64_t i = 0; i < nS; i++)
            if (v->S_flag[i])
                for (uint64_t d = 0; d < 8; d++) w->S_key[j++] = (v->S_key[i] << 3) | d;
    }

    if (labels)
        for (int L = 1; L < h->nlev; L++)
            if (label_level(h, L, conn) != 0) goto oom;

    free(sorted); free(pcell); free(pidx);
    *out = h;
    return 0;
oom:
    free(ki); free(sorted); free(pcell); free(pidx);
    orc_free(h);
    return -3;
fail:
    free(sorted); free(pcell); free(pidx);
    orc_free(h);
    return -4;
}

/* -------------------------------------------------------- accessors */

int orc_num_levels(const orc_hier *h) { return h->nlev; }
const uint32_t *orc_order(const orc_hier *h) { return h->order; }

int orc_level_sizes(const orc_hier *h, int L, uint64_t *sz /* [5] */)
{
    if (L < 0 || L >= h->nlev) return -1;
    const orc_level *v = &h->lev[L];
    sz[0] = v->nS; sz[1] = v->nE; sz[2] = v->nP; sz[3] = v->npatch; sz[4] = (uint64_t)v->b;
    return 0;
}

int orc_level_cells(const orc_hier *h, int L, uint64_t *key, uint32_t *count,
                    uint32_t *start, uint8_t *flag, int32_t *patch, double *pmass)
{
    if (L < 0 || L >= h->nlev) return -1;
    const orc_level *v = &h->lev[L];
    for (uint64_t i = 0; i < v->nS; i++) {
        key[i] = v->S_key[i];
        count[i] = v->S_count[i];
        start[i] = v->S_start[i];
        flag[i] = v->S_flag[i];
        patch[i] = v->S_patch ? v->S_patch[i] : -1;
        pmass[i] = v->S_pmass[i];
    }
    return 0;
}

int orc_level_field(const orc_hier *h, int L, uint64_t *key, double *m, uint8_t *ghost)
{
    if (L < 0 || L >= h->nlev) return -1;
    const orc_level *v = &h->lev[L];
    for (uint64_t e = 0; e < v->nE; e++) {
        key[e] = v->E_key[e];
        m[e] = v->E_mass[e];
        ghost[e] = v->E_ghost[e];
    }
    return 0;
}

int orc_level_totals(const orc_hier *h, int L, double *tot /* [2] */)
{
    if (L < 0 || L >= h->nlev) return -1;
    tot[0] = h->lev[L].tot_cell_mass;
    tot[1] = h->lev[L].tot_part_mass;
    return 0;
}

int orc_level_patches(const orc_hier *h, int L, int32_t *parent, uint64_t *ncells,
                      uint64_t *npart, double *pm)
{
    if (L < 0 || L >= h->nlev) return -1;
    const orc_level *v = &h->lev[L];
    for (uint64_t p = 0; p < v->npatch; p++) {
        parent[p] = v->patch_parent[p];
        ncells[p] = v->patch_ncells[p];
        npart[p] = v->patch_npart[p];
        pm[p] = v->patch_mass[p];
    }
    return 0;
}

/* ------------------------------------------------------------ probe */
/*
 * Single-cell questions answered straight from the definition, for checking
 * sampled cells of inputs too large for orc_build.  A cell c of level L is in
 * S_L iff every ancestor on levels 0..L-1 holds more particles than its
 * level's threshold (and those levels are below the level cap); its count is
 * the number of particles inside it; its field value is the TSC sum over the
 * particles of the S_L cells within one cell of it.
 */
typedef struct {
    uint64_t n;
    int g, B, max_levels;
    double dom_ref, ref_ref, mass_scalar;
    uint64_t *key;      /* sorted B-bit keys */
    uint32_t *idx;      /* input index of each sorted particle */
    const uint32_t *X, *Y, *Z;
    const float *fx, *fy, *fz, *mass;
} orc_probe;

orc_probe *orc_probe_create(uint64_t n, const uint32_t *X, const uint32_t *Y, const uint32_t *Z,
                            const float *fx, const float *fy, const float *fz, const float *mass,
                            double mass_scalar, int g, double dom_ref, double ref_ref, int max_levels)
{
    if (g < 1 || max_levels < 0 || g + max_levels > 21) return NULL;
    orc_probe *q = (orc_probe *)calloc(1, sizeof(orc_probe));
    keyidx *ki = (keyidx *)malloc(sizeof(keyidx) * (n ? n : 1));
    if (!q || !ki) { free(q); free(ki); return NULL; }
    q->n = n; q->g = g; q->B = g + max_levels; q->max_levels = max_levels;
    q->dom_ref = dom_ref; q->ref_ref = ref_ref; q->mass_scalar = mass_scalar;
    q->X = X; q->Y = Y; q->Z = Z; q->fx = fx; q->fy = fy; q->fz = fz; q->mass = mass;
    int B = q->B;
    for (uint64_t p = 0; p < n; p++) {
        ki[p].key = morton(X[p] >> (21 - B), Y[p] >> (21 - B), Z[p] >> (21 - B), B);
        ki[p].idx = (uint32_t)p;
    }
    qsort(ki, n, sizeof(keyidx), cmp_keyidx);
    q->key = (uint64_t *)malloc(sizeof(uint64_t) * (n ? n : 1));
    q->idx = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
    if (!q->key || !q->idx) { free(ki); free(q->key); free(q->idx); free(q); return NULL; }
    for (uint64_t p = 0; p < n; p++) { q->key[p] = ki[p].key; q->idx[p] = ki[p].idx; }
    free(ki);
    return q;
}

void orc_probe_free(orc_probe *q)
{
    if (!q) return;
    free(q->key); free(q->idx); free(q);
}

/* particles of the level-L cell with key k occupy sorted positions [*lo, *hi) */
static void probe_range(const orc_probe *q, int L, uint64_t k, uint64_t *lo, uint64_t *hi)
{
    int sh = 3 * (q->B - (q->g + L));
    *lo = lower_bound(q->key, q->n, k << sh);
    *hi = lower_bound(q->key, q->n, (k + 1) << sh);
}

static int probe_in_S(const orc_probe *q, int L, uint64_t k)
{
    if (L > q->max_levels) return 0;
    for (int l = 0; l < L; l++) {
        uint64_t a = k >> (3 * (L - l));
        uint64_t lo, hi;
        probe_range(q, l, a, &lo, &hi);
        double thr = (l == 0) ? q->dom_ref : q->ref_ref;
        if (!((double)(hi - lo) > thr)) return 0;
    }
    return 1;
}

/*
 * out[0] = 1 if the cell is in S_L, out[1] = 1 if it is in E_L,
 * out[2] = count, out[3] = start (global order), out[4] = refined flag;
 * *m = TSC mass of the cell (0 if outside E_L).
 */
int orc_probe_cell(const orc_probe *q, int L, uint64_t k, int64_t *out, double *m)
{
    int b = q->g + L;
    if (L < 0 || L > q->max_levels) return -1;
    uint64_t lo, hi;
    int inS = probe_in_S(q, L, k);
    probe_range(q, L, k, &lo, &hi);
    out[0] = inS;
    out[2] = (int64_t)(hi - lo);
    out[3] = (int64_t)lo;
    double thr = (L == 0) ? q->dom_ref : q->ref_ref;
    out[4] = inS && L < q->max_levels && b < 21 && (double)(hi - lo) > thr;
    int inE = 0;
    double acc = 0.0;
    for (int dx = -1; dx <= 1; dx++)
        for (int dy = -1; dy <= 1; dy++)
            for (int dz = -1; dz <= 1; dz++) {
                uint64_t s = neighbour(k, b, dx, dy, dz);
                if (!probe_in_S(q, L, s)) continue;
                inE = 1;
                uint64_t a, e;
                probe_range(q, L, s, &a, &e);
                for (uint64_t i = a; i < e; i++) {
                    uint32_t p = q->idx[i];
                    double mp = q->mass ? (double)q->mass[p] : q->mass_scalar;
                    /* the particle sits in cell s; cell k is at offset -(dx,dy,dz) from it */
                    double w = tsc_weight(-dx, in_cell(q->X[p], q->fx[p], b)) *
                               tsc_weight(-dy, in_cell(q->Y[p], q->fy[p], b)) *
                               tsc_weight(-dz, in_cell(q->Z[p], q->fz[p], b));
                    acc += mp * w;
                }
            }
    out[1] = inE;
    *m = acc;
    return 0;
}

uint64_t orc_morton(uint32_t x, uint32_t y, uint32_t z, int bits) { return morton(x, y, z, bits); }
