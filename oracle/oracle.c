/*
 * Race-check oracle: test infrastructure only.
 *
 * Plain, slow, single-threaded CPU code that decides which memory locations
 * of an access log take part in a data race.  It shares no code with the HIP
 * checker and is called only from the tests, the smoke check and the CPU
 * baseline leg of the benchmark.
 *
 * Definition followed (paper, Sec. II-A "Data Races" and Sec. II-B "CUDA
 * Shared-Memory Concurrency"): two accesses to the same location race when
 * they come from different threads, at least one of them conflicts with the
 * other, and no happens-before relation orders them.  Happens-before here is
 * generated only by
 *   - kernel launch boundaries (every access of launch L precedes every
 *     access of launch L+1 of the same job),
 *   - block-scope barriers (within one block, an access in block-barrier
 *     epoch e precedes every access in a later epoch; Sec. III-A, Scenario 2:
 *     a differing block clock BC means "block-synchronised"),
 *   - wave-scope barriers (within one wave and one block epoch, an access in
 *     wave-barrier epoch e precedes every access in a later wave epoch;
 *     Sec. III-B "Further Extension", warp-scope barriers with a warp clock WC),
 *   - optionally, tile barriers nested in the waves (synchronization of groups
 *     below a warp, which the paper leaves as future work, Sec. VI): within
 *     one tile of tile_width lanes, one block epoch and one wave epoch, an
 *     access in tile-barrier epoch e precedes every access in a later tile
 *     epoch.  A wave barrier restarts the tile epochs, as a block barrier
 *     restarts the wave epochs.
 * Atomics are a third class of access (Sec. III-B): two atomics never race
 * with each other, an atomic and a plain read or write do.  Atomics and
 * fences create no happens-before.  Lanes of one wave are not ordered by
 * lockstep execution; only barriers order them.
 *
 * Everything here is plain: records are sorted by location, and for every
 * location and launch the conflict-capable pairs (a write against any other
 * access, a plain read against an atomic) are tested one by one.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { K_READ = 0, K_WRITE = 1, K_ATOMIC = 2 };
enum { SP_GLOBAL = 0, SP_LDS = 1 };

typedef struct {
    uint64_t index;      /* element index within the region */
    uint32_t space;      /* SP_GLOBAL or SP_LDS */
    uint32_t region;     /* region (array) id within the space */
    uint32_t lds_block;  /* owning block of an LDS location, 0 for global */
    uint32_t kind;       /* K_READ, K_WRITE or K_ATOMIC */
    uint32_t launch;     /* launch sequence number within the job */
    uint32_t block;      /* linear block id of the accessing thread */
    uint32_t thread;     /* linear thread id within the block */
    uint32_t bc;         /* block-barrier epoch of the accessing thread */
    uint32_t wc;         /* wave-barrier epoch (reset at each block barrier) */
    uint32_t tc;         /* tile-barrier epoch (reset at each wave or block barrier) */
} orc_rec;               /* 48 bytes */

typedef struct {
    uint64_t index;
    uint32_t space, region, lds_block, pad;
} orc_key;               /* 24 bytes */

/* ---------------------------------------------------------------------- */
/* The pairwise predicate (Sec. II-A definition; Sec. II-B scopes).        */
/* ---------------------------------------------------------------------- */
int orc_race_pair_nested(const orc_rec* p, const orc_rec* c, uint32_t wave_width,
                         uint32_t tile_width)
{
    /* different threads */
    if (p->block == c->block && p->thread == c->thread) return 0;
    /* conflicting: not both plain reads, not both atomics */
    if (p->kind == c->kind && p->kind != K_WRITE) return 0;
    /* ordered by a launch boundary */
    if (p->launch != c->launch) return 0;
    if (p->block == c->block) {
        /* ordered by a block barrier */
        if (p->bc != c->bc) return 0;
        if (p->thread / wave_width == c->thread / wave_width) {
            /* ordered by a wave barrier: same wave, same block epoch */
            if (p->wc != c->wc) return 0;
            /* ordered by a tile barrier: same tile, same wave epoch */
            if (tile_width && p->thread / tile_width == c->thread / tile_width &&
                p->tc != c->tc)
                return 0;
        }
    }
    return 1;
}

int orc_race_pair(const orc_rec* p, const orc_rec* c, uint32_t wave_width)
{
    return orc_race_pair_nested(p, c, wave_width, 0);
}

static int cmp_loc(const orc_rec* a, const orc_rec* b)
{
    if (a->space != b->space) return a->space < b->space ? -1 : 1;
    if (a->region != b->region) return a->region < b->region ? -1 : 1;
    if (a->lds_block != b->lds_block) return a->lds_block < b->lds_block ? -1 : 1;
    if (a->index != b->index) return a->index < b->index ? -1 : 1;
    return 0;
}

static int cmp_rec(const void* x, const void* y)
{
    const orc_rec* a = (const orc_rec*)x;
    const orc_rec* b = (const orc_rec*)y;
    int c = cmp_loc(a, b);
    if (c) return c;
    if (a->launch != b->launch) return a->launch < b->launch ? -1 : 1;
    return 0;
}

/* Does the group recs[0..n) (one location, one launch) hold a racing pair? */
static int group_races(const orc_rec* g, size_t n, uint32_t wave_width, uint32_t tile_width,
                       size_t* scratch_w, size_t* scratch_r, size_t* scratch_a)
{
    size_t nw = 0, nr = 0, na = 0;
    for (size_t i = 0; i < n; ++i) {
        if (g[i].kind == K_WRITE) scratch_w[nw++] = i;
        else if (g[i].kind == K_READ) scratch_r[nr++] = i;
        else scratch_a[na++] = i;
    }
    /* a write against every other access */
    for (size_t i = 0; i < nw; ++i)
        for (size_t j = 0; j < n; ++j)
            if (j != scratch_w[i] &&
                orc_race_pair_nested(&g[scratch_w[i]], &g[j], wave_width, tile_width))
                return 1;
    /* a plain read against an atomic */
    for (size_t i = 0; i < nr; ++i)
        for (size_t j = 0; j < na; ++j)
            if (orc_race_pair_nested(&g[scratch_r[i]], &g[scratch_a[j]], wave_width, tile_width))
                return 1;
    return 0;
}

/*
 * Flagged locations of an access log.  Sorts recs in place.  Writes the
 * sorted, unique racy keys to out (up to cap) and their count to *n_out.
 * Returns 0, or -1 when out is too small (then *n_out holds the needed count).
 */
int orc_flagged_nested(orc_rec* recs, size_t n, uint32_t wave_width, uint32_t tile_width,
                       orc_key* out, size_t cap, size_t* n_out)
{
    if (wave_width == 0) wave_width = 64;
    qsort(recs, n, sizeof(orc_rec), cmp_rec);
    size_t maxg = 0;   /* largest location group: bounds every launch group */
    for (size_t i = 0; i < n;) {
        size_t j = i + 1;
        while (j < n && cmp_loc(&recs[i], &recs[j]) == 0) ++j;
        if (j - i > maxg) maxg = j - i;
        i = j;
    }
    size_t* sw = (size_t*)malloc((maxg + 1) * sizeof(size_t));
    size_t* sr = (size_t*)malloc((maxg + 1) * sizeof(size_t));
    size_t* sa = (size_t*)malloc((maxg + 1) * sizeof(size_t));
    size_t found = 0;
    int rc = 0;
    for (size_t i = 0; i < n;) {
        /* one location: [i, k) */
        size_t k = i + 1;
        while (k < n && cmp_loc(&recs[i], &recs[k]) == 0) ++k;
        int racy = 0;
        for (size_t a = i; a < k && !racy;) {
            size_t b = a + 1;
            while (b < k && recs[b].launch == recs[a].launch) ++b;
            racy = group_races(&recs[a], b - a, wave_width, tile_width, sw, sr, sa);
            a = b;
        }
        if (racy) {
            if (found < cap && out) {
                out[found].index = recs[i].index;
                out[found].space = recs[i].space;
                out[found].region = recs[i].region;
                out[found].lds_block = recs[i].lds_block;
                out[found].pad = 0;
            }
            ++found;
        }
        i = k;
    }
    free(sw); free(sr); free(sa);
    if (found > cap) rc = -1;
    *n_out = found;
    return rc;
}

int orc_flagged(orc_rec* recs, size_t n, uint32_t wave_width,
                orc_key* out, size_t cap, size_t* n_out)
{
    return orc_flagged_nested(recs, n, wave_width, 0, out, cap, n_out);
}

/* ---------------------------------------------------------------------- */
/* Access-log models of the workloads.  Each walks the workload's program  */
/* thread by thread and emits one record per instrumented access, with the */
/* thread's block and wave barrier epochs.  With out == NULL they count.   */
/* ---------------------------------------------------------------------- */
typedef struct {
    orc_rec* out;
    size_t cap, n;
} sink;

static void emit_tc(sink* s, uint32_t space, uint32_t region, uint64_t index,
                    uint32_t kind, uint32_t launch, uint32_t block,
                    uint32_t thread, uint32_t bc, uint32_t wc, uint32_t tc)
{
    if (s->out && s->n < s->cap) {
        orc_rec* r = &s->out[s->n];
        r->index = index;
        r->space = space;
        r->region = region;
        r->lds_block = space == SP_LDS ? block : 0;
        r->kind = kind;
        r->launch = launch;
        r->block = block;
        r->thread = thread;
        r->bc = bc;
        r->wc = wc;
        r->tc = tc;
    }
    s->n++;
}

static void emit(sink* s, uint32_t space, uint32_t region, uint64_t index,
                 uint32_t kind, uint32_t launch, uint32_t block,
                 uint32_t thread, uint32_t bc, uint32_t wc)
{
    emit_tc(s, space, region, index, kind, launch, block, thread, bc, wc, 0);
}

/*
 * LDS tree reduction: each of `blocks` blocks of T threads sums n int32
 * words (n a power of two, n <= 2T).  Thread t loads words t, t+T, ... of
 * its block's slice; when n != 2T a block barrier follows the loads (a
 * thread's first operand then comes from another thread).  Step s
 * (h = n >> (s+1)): threads t < h read a[t] and a[t+h] and write a[t]; a
 * block barrier follows unless s == drop.  Every thread then reads a[0] and
 * writes out[b*T + t].  Global region 0 = in, 1 = out; LDS array 0 = a.
 * The paper-sized case is n = 512, T = 256, one block.
 */
size_t orc_model_reduce_n(uint32_t n, uint32_t T, uint32_t blocks, int drop, uint32_t launch,
                          orc_rec* out, size_t cap)
{
    sink s = {out, cap, 0};
    uint32_t steps = 0;
    while ((1u << steps) < n) ++steps;
    for (uint32_t b = 0; b < blocks; ++b) {
        for (uint32_t t = 0; t < T; ++t) {
            uint32_t bc = 0;
            for (uint32_t j = t; j < n; j += T) {
                emit(&s, SP_GLOBAL, 0, (uint64_t)b * n + j, K_READ, launch, b, t, bc, 0);
                emit(&s, SP_LDS, 0, j, K_WRITE, launch, b, t, bc, 0);
            }
            if (n != 2 * T) ++bc;
            for (uint32_t step = 0; step < steps; ++step) {
                const uint32_t h = n >> (step + 1);
                if (t < h) {
                    emit(&s, SP_LDS, 0, t, K_READ, launch, b, t, bc, 0);
                    emit(&s, SP_LDS, 0, t + h, K_READ, launch, b, t, bc, 0);
                    emit(&s, SP_LDS, 0, t, K_WRITE, launch, b, t, bc, 0);
                }
                if ((int)step != drop) ++bc;
            }
            emit(&s, SP_LDS, 0, 0, K_READ, launch, b, t, bc, 0);
            emit(&s, SP_GLOBAL, 1, (uint64_t)b * T + t, K_WRITE, launch, b, t, bc, 0);
        }
    }
    return s.n;
}

/* The paper-sized reduction: 512 words, 256 threads, one block. */
size_t orc_model_reduce(int drop, uint32_t launch, orc_rec* out, size_t cap)
{
    return orc_model_reduce_n(512, 256, 1, drop, launch, out, cap);
}

/*
 * 5-point Jacobi sweep on an ny x nx grid with 16x16-thread blocks and an
 * 18x18 LDS tile (halo ring, corners unused).  Launch L reads region L%2 and
 * writes region (L+1)%2.  Only blocks with bx in [bx0,bx1) and by in
 * [by0,by1) are modelled.  seed_tab[block] is -1 or (side<<8 | offset): that
 * block's edge thread next to the halo cell (side, offset) also writes that
 * neighbour-owned cell of the output array (sides: 0 N, 1 S, 2 W, 3 E).
 */
size_t orc_model_jacobi(uint32_t ny, uint32_t nx, uint32_t launch0,
                        uint32_t launches, const int32_t* seed_tab,
                        uint32_t bx0, uint32_t bx1, uint32_t by0, uint32_t by1,
                        orc_rec* out, size_t cap)
{
    sink s = {out, cap, 0};
    const uint32_t nbx = (nx + 15) / 16;
    for (uint32_t L = launch0; L < launch0 + launches; ++L) {
        const uint32_t rin = L % 2, rout = (L + 1) % 2;
        for (uint32_t by = by0; by < by1; ++by)
        for (uint32_t bx = bx0; bx < bx1; ++bx) {
            const uint32_t b = by * nbx + bx;
            const int32_t sd = seed_tab ? seed_tab[b] : -1;
            for (uint32_t t = 0; t < 256; ++t) {
                const uint32_t tx = t % 16, ty = t / 16;
                const uint32_t gx = bx * 16 + tx, gy = by * 16 + ty;
                if (gx >= nx || gy >= ny) continue;
                const uint64_t g = (uint64_t)gy * nx + gx;
                const uint32_t cl = (ty + 1) * 18 + tx + 1;
                /* staging into LDS, block epoch 0 */
                emit(&s, SP_GLOBAL, rin, g, K_READ, L, b, t, 0, 0);
                emit(&s, SP_LDS, 0, cl, K_WRITE, L, b, t, 0, 0);
                if (ty == 0 && gy > 0) {
                    emit(&s, SP_GLOBAL, rin, g - nx, K_READ, L, b, t, 0, 0);
                    emit(&s, SP_LDS, 0, tx + 1, K_WRITE, L, b, t, 0, 0);
                }
                if (ty == 15 && gy + 1 < ny) {
                    emit(&s, SP_GLOBAL, rin, g + nx, K_READ, L, b, t, 0, 0);
                    emit(&s, SP_LDS, 0, 17 * 18 + tx + 1, K_WRITE, L, b, t, 0, 0);
                }
                if (tx == 0 && gx > 0) {
                    emit(&s, SP_GLOBAL, rin, g - 1, K_READ, L, b, t, 0, 0);
                    emit(&s, SP_LDS, 0, (ty + 1) * 18, K_WRITE, L, b, t, 0, 0);
                }
                if (tx == 15 && gx + 1 < nx) {
                    emit(&s, SP_GLOBAL, rin, g + 1, K_READ, L, b, t, 0, 0);
                    emit(&s, SP_LDS, 0, (ty + 1) * 18 + 17, K_WRITE, L, b, t, 0, 0);
                }
                /* block barrier, then the 5-point update in block epoch 1 */
                emit(&s, SP_LDS, 0, cl, K_READ, L, b, t, 1, 0);
                if (gy > 0) emit(&s, SP_LDS, 0, cl - 18, K_READ, L, b, t, 1, 0);
                if (gy + 1 < ny) emit(&s, SP_LDS, 0, cl + 18, K_READ, L, b, t, 1, 0);
                if (gx > 0) emit(&s, SP_LDS, 0, cl - 1, K_READ, L, b, t, 1, 0);
                if (gx + 1 < nx) emit(&s, SP_LDS, 0, cl + 1, K_READ, L, b, t, 1, 0);
                emit(&s, SP_GLOBAL, rout, g, K_WRITE, L, b, t, 1, 0);
                if (sd >= 0) {
                    const uint32_t side = (uint32_t)sd >> 8, off = (uint32_t)sd & 255;
                    int64_t tgt = -1;
                    if (side == 0 && ty == 0 && tx == off) tgt = (int64_t)g - nx;
                    if (side == 1 && ty == 15 && tx == off) tgt = (int64_t)g + nx;
                    if (side == 2 && tx == 0 && ty == off) tgt = (int64_t)g - 1;
                    if (side == 3 && tx == 15 && ty == off) tgt = (int64_t)g + 1;
                    if (tgt >= 0)
                        emit(&s, SP_GLOBAL, rout, (uint64_t)tgt, K_WRITE, L, b, t, 1, 0);
                }
            }
        }
    }
    return s.n;
}

/*
 * Label propagation, one thread per vertex v (block v / tpb, thread v % tpb):
 * an atomic load of label[v], then for every out-edge e = (v, u) an atomic
 * min into label[u]; a seeded edge (mask[e] != 0) instead does a plain read
 * and a plain write of label[u].  Region 0 = label[n].  With monitor_csr the
 * reads of row_ptr (region 1) and col (region 2) are logged as well.
 * When keep != NULL only records whose label index u has keep[u] != 0 are
 * emitted (CSR records are then dropped).
 */
size_t orc_model_labelprop(uint32_t n, const int32_t* row_ptr, const int32_t* col,
                           const uint8_t* mask, uint32_t launch0, uint32_t launches,
                           uint32_t tpb, int monitor_csr, const uint8_t* keep,
                           orc_rec* out, size_t cap)
{
    sink s = {out, cap, 0};
    for (uint32_t L = launch0; L < launch0 + launches; ++L) {
        for (uint32_t v = 0; v < n; ++v) {
            const uint32_t b = v / tpb, t = v % tpb;
            if (!keep || keep[v])
                emit(&s, SP_GLOBAL, 0, v, K_ATOMIC, L, b, t, 0, 0);
            if (monitor_csr && !keep) {
                emit(&s, SP_GLOBAL, 1, v, K_READ, L, b, t, 0, 0);
                emit(&s, SP_GLOBAL, 1, v + 1, K_READ, L, b, t, 0, 0);
            }
            for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
                const uint32_t u = (uint32_t)col[e];
                if (monitor_csr && !keep)
                    emit(&s, SP_GLOBAL, 2, (uint64_t)e, K_READ, L, b, t, 0, 0);
                if (keep && !keep[u]) continue;
                if (mask[e]) {
                    emit(&s, SP_GLOBAL, 0, u, K_READ, L, b, t, 0, 0);
                    emit(&s, SP_GLOBAL, 0, u, K_WRITE, L, b, t, 0, 0);
                } else {
                    emit(&s, SP_GLOBAL, 0, u, K_ATOMIC, L, b, t, 0, 0);
                }
            }
        }
    }
    return s.n;
}

/*
 * One launch of an interpreted barrier program (layout documented with the
 * program generator): per phase, every thread's operations, then the phase's
 * barrier.  A block barrier advances the block epoch and restarts the wave
 * and tile epochs; a wave barrier advances the wave epoch of the waves in
 * wave_mask and restarts their tile epochs; a tile barrier (scope 3, with
 * tile_width lanes per tile) advances the tile epoch of the tiles in the
 * mask.  An operation of kind 3 switches the thread's monitoring off (index
 * bit 0 clear) or on (set): the accesses a switched-off thread makes are not
 * monitored, so they are not in the log (paper Sec. IV-A: the instrumentation
 * of individual threads can be enabled or disabled at run time).
 */
size_t orc_model_launch_nested(uint32_t launch, uint32_t blocks, uint32_t threads,
                               uint32_t phases, const uint8_t* scope,
                               const uint64_t* wave_mask, const int32_t* op_off,
                               const uint32_t* ops, uint32_t wave_width, uint32_t tile_width,
                               orc_rec* out, size_t cap)
{
    sink s = {out, cap, 0};
    if (wave_width == 0) wave_width = 64;
    for (uint32_t b = 0; b < blocks; ++b) {
        for (uint32_t t = 0; t < threads; ++t) {
            uint32_t bc = 0, wc = 0, tc = 0, on = 1;
            const uint32_t w = t / wave_width;
            const uint32_t g = tile_width ? t / tile_width : 0;
            for (uint32_t p = 0; p < phases; ++p) {
                const size_t i = ((size_t)p * blocks + b) * threads + t;
                for (int32_t k = op_off[i]; k < op_off[i + 1]; ++k) {
                    const uint32_t op = ops[k];
                    if (((op >> 27) & 3) == 3) {
                        on = op & 1;
                        continue;
                    }
                    if (on)
                        emit_tc(&s, (op >> 29) & 1, (op >> 24) & 7, op & 0xFFFFFF,
                                (op >> 27) & 3, launch, b, t, bc, wc, tc);
                }
                if (scope[p] == 2) { ++bc; wc = 0; tc = 0; }
                else if (scope[p] == 1 && w < 64 && ((wave_mask[p] >> w) & 1)) { ++wc; tc = 0; }
                else if (scope[p] == 3 && tile_width && g < 64 && ((wave_mask[p] >> g) & 1)) ++tc;
            }
        }
    }
    return s.n;
}

size_t orc_model_launch(uint32_t launch, uint32_t blocks, uint32_t threads,
                        uint32_t phases, const uint8_t* scope,
                        const uint64_t* wave_mask, const int32_t* op_off,
                        const uint32_t* ops, uint32_t wave_width,
                        orc_rec* out, size_t cap)
{
    return orc_model_launch_nested(launch, blocks, threads, phases, scope, wave_mask, op_off,
                                   ops, wave_width, 0, out, cap);
}
