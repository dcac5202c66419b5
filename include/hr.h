/*
 * hr.h -- C ABI of the MI355X (gfx950) race checker.
 *
 * The checker follows HiRace (Jacobson, Burtscher, Gopalakrishnan): every
 * monitored 4-byte element of global memory or LDS has a constant-size
 * shadow word holding a per-location state machine; each instrumented access
 * advances it with a compare-and-swap (paper Sec. IV-B, Algorithm 1), and a
 * transition into the race state is appended once to a report ring
 * (Sec. V-C reports races on unique addresses).  Races are the paper's
 * (Sec. II-A): same location, different threads, at least one write (or a
 * plain access meeting an atomic, Sec. III-B), not ordered by a launch
 * boundary, a block barrier or a wave barrier (Sec. II-B).
 *
 * Conventions for every call:
 *  - Pointers named *_dev are device pointers (HIP device memory); all other
 *    pointers are host pointers.  The caller owns its data buffers and
 *    streams; a context owns its shadow memory, report ring and counters.
 *  - `stream` is a hipStream_t passed as void*; NULL means the stream given
 *    to hr_ctx_create.  Calls are stream-ordered and asynchronous unless
 *    stated otherwise.
 *  - Negative status: error, nothing was changed.  Positive status: a bit set
 *    of warnings; results gathered so far remain valid.
 *  - The caller serialises calls on one context (no internal locking).
 */
#ifndef HR_H
#define HR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hr_ctx_s* hr_ctx;

typedef enum {
    HR_OK = 0,
    /* Warnings (bit set).  Clock overflow: a block or wave clock passed its
     * configured width; checking stopped in the affected threads after the
     * races found so far were recorded (paper Sec. III-A, footnote on clock
     * sizes). */
    HR_W_CLOCK_OVERFLOW = 1,
    /* More races than ring slots; hr_report then completes the global-memory
     * part of the set from the sticky race states in shadow memory, while LDS
     * races beyond the ring are lost. */
    HR_W_RING_OVERFLOW = 2,
    /* An instrumented access named an element outside its region; it was
     * neither checked nor performed by the library's own kernels. */
    HR_W_OUT_OF_RANGE = 4,
    /* A batched work item waited too long for the previous phase of its job
     * and was skipped, or a tile of a served large stencil job waited too
     * long at its barrier and went on; that job's results are incomplete. */
    HR_W_STALLED = 8,
    /* Some call site reached hr_config.site_limit: its further race records
     * were dropped.  hr_report still completes the global-memory part of the
     * set from the sticky race states in shadow memory; LDS races whose
     * records were dropped are lost. */
    HR_W_REPORT_LIMITED = 16,
    /* HR_CFG_WORD4 only: some checked thread's block id or thread index did
     * not fit the 4-byte word's block or thread field, so ids were taken
     * modulo the field widths; races between accessors whose ids fold
     * together may be missing from the set (none is ever invented). */
    HR_W_FOLDED = 32,
    /* HR_CFG_ACCESS_LOG only: more accesses than log_capacity; the log holds
     * the first log_capacity of them (in no particular order). */
    HR_W_LOG_TRUNCATED = 64,
    /* A masked wave barrier (__syncwarp(mask) in an instrumented kernel)
     * named only part of its caller's synchronization group (tile, or wave
     * when wave_bits is 6): it was not taken as ordering anything, so the
     * set may hold races that the barrier prevents (none is missed). */
    HR_W_PARTIAL_BARRIER = 128,
    HR_E_INVAL = -1,   /* bad argument */
    HR_E_NOMEM = -2,   /* allocation failed or shadow budget exceeded */
    HR_E_HIP = -3,     /* a HIP runtime call failed */
    HR_E_STATE = -4    /* call not valid in the context's current state */
} hr_status;

typedef enum { HR_GLOBAL = 0, HR_LDS = 1 } hr_space;
/* An atomic load counts as HR_ATOMIC: atomics are the third access class of
 * the paper's state machine (Sec. III-B). */
typedef enum { HR_READ = 0, HR_WRITE = 1, HR_ATOMIC = 2 } hr_kind;

/* Configuration of a context.  The paper exposes the checker's settings as a
 * configuration, among them bounds on the shadow metadata that trade memory
 * for range (Sec. IV, introduction), and makes the scalar clocks' widths
 * configurable, with checking stopped by a warning when a clock overflows
 * (Sec. III-A, footnote on clock sizes).  Zero fields take the defaults. */
typedef struct {
    uint32_t ring_capacity;  /* race records kept on the device; 0: 65536 */
    uint32_t bc_bits;        /* block-clock width 1..8; 0: 8 (HR_CFG_WORD4: 2) */
    uint32_t wc_bits;        /* wave-clock width 1..6; 0: 6 (HR_CFG_WORD4: 1) */
    uint32_t flags;          /* HR_CFG_* bits */
    uint64_t shadow_budget;  /* cap on shadow bytes of this context; 0: none */
    uint32_t site_limit;     /* race records kept per call site (site id mod
                                HR_SITES) between two hr_reset calls; 0: no
                                limit.  Past it, records of that site are
                                dropped and hr_report warns
                                HR_W_REPORT_LIMITED.  The batched and serving
                                executors do not apply it. */
    uint32_t wave_bits;      /* lanes of the wave-scope synchronization group,
                                log2: 6 (0 means 6) for whole waves, 1..5 for
                                aligned tiles of 2^wave_bits lanes; then every
                                wave-scope barrier of the job is a tile
                                barrier (a tiled partition's sync) and orders
                                only its tile's lanes.  Wave grouping of hook
                                lanes only runs with whole waves.  With
                                HR_CFG_NESTED_TILES: the tiles nested in the
                                waves (1..5). */
    uint32_t thread_bits;    /* HR_CFG_WORD4 only: width of the thread field,
                                1..10; 0: 8.  The block field gets the rest,
                                27 - wc_bits - bc_bits - thread_bits bits
                                (3 to 22; 16 with the defaults). */
    uint32_t coalesce_width; /* with HR_CFG_WAVE_GROUPING: lanes are grouped
                                within aligned segments of this many lanes
                                (a power of two, 2..64); 0: 64, the whole
                                wave.  Must be 0 without the flag. */
    uint32_t log_capacity;   /* with HR_CFG_ACCESS_LOG: access records kept on
                                the device, at most 2^28; 0: 2^20.  Must be 0
                                without the flag. */
    uint32_t pad;
} hr_config;

#define HR_SITES 256   /* call-site counters of the report limit */

/* Count every checked access in a device counter (read by hr_check_count). */
#define HR_CFG_COUNT_CHECKS 1u
/* Wave grouping at hook sites with data-dependent addresses: lanes of one
 * hook instruction that hit the same shadow word are folded into one update
 * by an owner lane (the result is unchanged; only the number of atomics
 * drops under same-word contention).  Off by default. */
#define HR_CFG_WAVE_GROUPING 2u
/* 4-byte global shadow words instead of 8-byte ones (the paper sizes its
 * shadow word by configuration, Sec. IV-A, and leaves footprint trade-offs
 * to the user): half the shadow memory.  The word holds the state number
 * (5 bits), the wave clock, the block clock, the thread and the block, of
 * the configured widths; it has no launch field, so hr_kernel_end returns
 * every word to the initial state at each launch boundary.  Exact while a
 * launch has at most 2^K blocks (K the block field's width) and 2^thread_bits
 * threads per block; beyond that, block ids and thread indices are taken
 * modulo those powers, races between accessors that then look alike can be
 * missed (never invented), and hr_report warns HR_W_FOLDED.  Race records carry 8-byte summaries with
 * launch 0 and the folded block.  The batched and serving executors reject
 * such a context. */
#define HR_CFG_WORD4 4u
/* Debug: every hook also appends the access it checks to a bounded device
 * log (hr_access_log), so that the accesses the checker saw can be compared
 * one by one with a model of the program.  Implies HR_CFG_COUNT_CHECKS. */
#define HR_CFG_ACCESS_LOG 8u
/* Tiles nested in waves: the synchronization below the warp that the paper
 * leaves to future work (Sec. VI), as cooperative-groups tiles use it beside
 * wave barriers.  wave_bits = s (1..5, required) names aligned tiles of 2^s
 * lanes that have their own barrier; wave barriers still order whole waves.
 * Shadow words then carry a tile level and a tile clock (the nested machine;
 * block ids below 2^20, block clock width at most 5, wave clock width at
 * most 4, default 5 and 4, tile clock 4 bits).  The access-program
 * interpreter (hr_program_check, scope 3 = tile barrier) runs such jobs; the
 * other workloads, the batched and serving executors and hr_job_run_static
 * reject such a context.  Not with HR_CFG_WORD4 or HR_CFG_WAVE_GROUPING. */
#define HR_CFG_NESTED_TILES 16u
/* Global-word transitions read from the flat table of the state machine
 * (the paper's encoding, Sec. IV-B: an array indexed by the old state and
 * the transition labels) instead of computed by bit logic; the same machine
 * and the same results, at another cost, for the autotuner to time.  The
 * context holds the table (32 KiB) in device memory.  The stencil's checked
 * kernel (row-major maps) and the access-program interpreter honour it; the
 * other workloads, the executors and hr_job_run_static reject such a
 * context.  Not with HR_CFG_WORD4, HR_CFG_NESTED_TILES or HR_CFG_ACCESS_LOG. */
#define HR_CFG_FSM_TABLE 32u
/* As HR_CFG_FSM_TABLE (which it implies), with the stencil's checked kernel
 * reading the table from a copy in each block's LDS; the interpreter reads
 * the device-memory copy. */
#define HR_CFG_FSM_TABLE_LDS 64u

/* One flagged location, 48 bytes.  The key is (space, region, block if LDS,
 * index).  The other fields describe how the race was found: `before` and
 * `with` are two shadow summaries (global- or LDS-word layout, by space;
 * decode them with hr_describe, or hr_describe_nested in a context with
 * HR_CFG_NESTED_TILES) whose accesses include a racing pair.
 * `before` is the word the race state replaced.  `with` is the completing
 * access alone (a single-thread summary holding its launch, block, thread,
 * block clock, wave clock and class) or, for a record made while folding
 * back an overwritten update (HR_RACE_FOLD), the summary folded back. */
typedef struct {
    uint8_t space;          /* hr_space */
    uint8_t kind;           /* hr_kind of the access whose hook found the race */
    uint16_t site;          /* its call-site id (0: none given) */
    uint32_t region;        /* region id (global) or LDS array id */
    uint32_t block;         /* owning block (LDS) / block of that access (global) */
    uint32_t launch;        /* launch sequence number within the job */
    uint64_t index;         /* element index within the region */
    uint64_t before;        /* summary replaced by the race state */
    uint64_t with;          /* summary it met (see above) */
    uint32_t tid;           /* thread of that access within its block */
    uint32_t flags;         /* HR_RACE_* bits */
} hr_race;

#define HR_RACE_FOLD 1u      /* found while folding back an overwritten summary */
#define HR_RACE_SCANNED 2u   /* recovered by the ring-overflow scan: only the key is valid */

/* A shadow summary decoded (hr_describe).  Fields a state does not keep are
 * UINT32_MAX; classes are 1 (reads), 2 (atomics), 3 (a write, or reads and
 * atomics), 0 when not kept. */
typedef enum {
    HR_S_INIT = 0,          /* never accessed */
    HR_S_RACE = 1,          /* race state */
    HR_S_BLOCKS = 2,        /* accesses from >= 2 blocks, all of class_block */
    HR_S_WAVES = 3,         /* one block; >= 2 waves in its latest block epoch */
    HR_S_THREADS = 4,       /* one wave; >= 2 threads in its latest wave epoch */
    HR_S_THREAD = 5,        /* one thread in the latest wave epoch */
    HR_S_TILES = 6          /* tiles nested in waves: one wave; >= 2 tiles in its
                               latest wave epoch (hr_describe_nested) */
} hr_summary_state;

typedef struct {
    uint32_t state;         /* hr_summary_state */
    uint32_t class_launch;  /* class of the (single) block's accesses this launch */
    uint32_t class_block;   /* class in the latest block epoch (HR_S_BLOCKS: of all) */
    uint32_t class_wave;    /* class in the latest wave epoch */
    uint32_t launch;        /* launch epoch (global words; 9 bits) */
    uint32_t block, bc;     /* the block and its block clock */
    uint32_t wave, wc;      /* the wave (or tile) and its clock */
    uint32_t thread;        /* the thread (HR_S_THREAD) */
} hr_summary;

/* A shadow summary of a context with HR_CFG_NESTED_TILES decoded
 * (hr_describe_nested): waves of 64 lanes, each split into tiles with their
 * own barriers and clocks.  In it HR_S_THREADS means one tile with >= 2
 * threads in its latest tile epoch, HR_S_THREAD one thread in that epoch,
 * and HR_S_TILES one wave with >= 2 tiles in its latest wave epoch.  Fields
 * a state does not keep are UINT32_MAX, classes 0, as in hr_summary. */
typedef struct {
    uint32_t state;         /* hr_summary_state */
    uint32_t class_launch;  /* class of the (single) block's accesses this launch */
    uint32_t class_block;   /* class in the latest block epoch (HR_S_BLOCKS: of all) */
    uint32_t class_wave;    /* class in the latest wave epoch */
    uint32_t class_tile;    /* class in the latest tile epoch */
    uint32_t launch;        /* launch epoch (global words; 9 bits) */
    uint32_t block, bc;     /* the block and its block clock */
    uint32_t wave, wc;      /* the wave (thread / 64) and its wave clock */
    uint32_t tile, tc;      /* the tile (thread >> tile_bits) and its tile clock */
    uint32_t thread;        /* the thread (HR_S_THREAD) */
} hr_summary_nested;

/* Create a context whose default stream is `stream` (paper Sec. IV: the
 * checker's configuration; Sec. III-A, footnote on clock sizes: the clock
 * widths of cfg bound the block and wave clocks).  Allocates the report ring
 * and counters on the current HIP device; the context owns them and every
 * shadow region later allocated in it.  cfg may be NULL (defaults); it is
 * copied.  *out receives the context, or NULL on error.
 * Errors: HR_E_INVAL (out NULL, cfg out of range: unknown flags, bc_bits > 8,
 * wc_bits > 6, wave_bits > 6, ring_capacity > 2^26, thread_bits set without
 * HR_CFG_WORD4 or above 10, coalesce_width not 0 or a power of two in
 * 2..64, or set without HR_CFG_WAVE_GROUPING), HR_E_NOMEM (a device
 * allocation failed),
 * HR_E_HIP. */
hr_status hr_ctx_create(hr_ctx* out, const hr_config* cfg, void* stream);

/* Free every device allocation of the context: shadow regions, batch arenas,
 * report ring and counters (the tool allocates the metadata of the data it
 * monitors and frees it again, Sec. IV-C; here the context owns all of it,
 * while the monitored buffers and the streams stay the caller's).  Blocks
 * until its default stream is idle; c is invalid afterwards.  Errors:
 * HR_E_INVAL (c NULL), HR_E_HIP (the stream reported an error; the memory is
 * freed all the same). */
hr_status hr_ctx_destroy(hr_ctx c);

/* Monitor `bytes` of device memory at data_dev as 4-byte elements (the
 * shadow-per-element layout of paper Sec. III-A, Fig. 2): allocates an
 * 8-byte shadow word per element (4-byte with HR_CFG_WORD4; the budget
 * counts whole 8-byte units), owned by the context and cleared to the
 * initial state.  Returns the region id (0..15) in *region_out.
 * Errors: HR_E_INVAL (elem_bytes != 4, bytes not a multiple of 4, 16 regions
 * in use), HR_E_NOMEM (allocation failed or shadow budget exceeded). */
hr_status hr_shadow_alloc(hr_ctx c, const void* data_dev, size_t bytes, uint32_t elem_bytes,
                          uint32_t* region_out);

/* Largest tile side of a tiled shadow map, log2 (tiles up to 16 x 16). */
#define HR_TILE_LOG2_MAX 4u

/* Monitor a rows x cols row-major array of 4-byte elements at data_dev with
 * a tiled address-to-shadow map.  The paper keeps one shadow entry per
 * monitored element (Sec. III-A, Fig. 2) but leaves where it lives open;
 * here the shadow words of each tile of 2^tile_w_log2 columns by
 * 2^tile_h_log2 rows are consecutive, tiles in row-major order, so that a
 * 2-D access pattern whose lanes walk down a column (a stencil's west or
 * east halo) touches few shadow cache lines.  Element (r, c) has its word at
 * ((r >> th) * ceil(cols / 2^tw) + (c >> tw)) << (tw + th)
 *   | (r mod 2^th) << tw | (c mod 2^tw)
 * (tw, th the two logs); the array is padded to whole tiles in shadow memory
 * only.  Both logs 0 give the row-major map of hr_shadow_alloc.  Element
 * indices (hooks, race records) stay row-major: r * cols + c.  Owned by the
 * context and cleared to the initial state, as hr_shadow_alloc; the 2-D
 * workloads (hr_jacobi_check) need cols equal to their row width.
 * Errors: HR_E_INVAL (elem_bytes != 4, a zero side, a tile log above
 * HR_TILE_LOG2_MAX, 16 regions in use), HR_E_NOMEM. */
hr_status hr_shadow_alloc_2d(hr_ctx c, const void* data_dev, uint32_t rows, uint32_t cols,
                             uint32_t elem_bytes, uint32_t tile_w_log2, uint32_t tile_h_log2,
                             uint32_t* region_out);

/* Switch the monitoring of a region off (on = 0) or back on, for the
 * kernels launched afterwards (the paper lets a tool enable or disable the
 * instrumentation of individual data at run time, Sec. IV-A).  Hooks on an
 * unmonitored region do nothing; its shadow words keep their state, so
 * switching it on again resumes checking with the history it had.  Device
 * code switches individual threads with hr_thread_enable.  Errors:
 * HR_E_INVAL (unknown or freed region). */
hr_status hr_region_enable(hr_ctx c, uint32_t region, uint32_t on);

/* Release the shadow memory of a region made by hr_shadow_alloc (for
 * long-lived contexts whose jobs end at different times).  Synchronises the
 * context's stream.  Errors: HR_E_INVAL (unknown or freed region),
 * HR_E_STATE (the region is a view into a batch's shared allocation). */
hr_status hr_shadow_free(hr_ctx c, uint32_t region);

/* Copy the plain-old-data block that instrumented kernels receive into out
 * (host memory, cap bytes; *size_out, when not NULL, receives its size).  It
 * carries what the per-access update of Algorithm 1 (Sec. IV-B) takes
 * besides the thread's own identity and clocks: the shadow address of each
 * region (the update's sAddr comes from it and the element index), the
 * region sizes, the report ring and counters, the clock limits and the
 * current launch epoch.  Its env.nested field is 1 in a context made with
 * HR_CFG_NESTED_TILES: kernels must then check with the nested hooks
 * (hr_tn, hr_nested.h), as the instrumenter's launchers do.  The device
 * pointers in it stay owned by the context.
 * The block is valid until the next hr_kernel_end, hr_reset or region
 * change.  Errors: HR_E_INVAL (c NULL, out NULL, or cap too small: *size_out
 * still receives the size needed). */
hr_status hr_dev_args(hr_ctx c, void* out, size_t cap, size_t* size_out);

/* Mark a kernel-launch boundary: every access of the launches before it
 * happens before every access after it (Sec. II-B: threads of one grid
 * synchronize only through barriers; a later launch on the same stream
 * starts after the earlier one ends).  Call it after each checked launch,
 * on the launch's stream.  Errors: HR_E_INVAL (c NULL), HR_E_HIP.  Advances
 * the launch epoch; every
 * 512 launches it clears the shadow on `stream`.  Races already found stay
 * in the ring; if the ring has overflowed, the global races held in the
 * shadow are first read back and kept for hr_report.  Asynchronous, except
 * at those clears, where it synchronises `stream` to read the ring count.
 * With HR_CFG_WORD4 it clears the shadow at every call instead, on `stream`
 * and without synchronising: a word in the race state keeps it when the
 * ring has overflowed (the clear reads the ring count on the device). */
hr_status hr_kernel_end(hr_ctx c, void* stream);

/* Start a new job on the same regions: clear shadow memory, report ring,
 * counters and warnings, and restart the launch count.  Asynchronous. */
hr_status hr_reset(hr_ctx c, void* stream);

/* Synchronise `stream`, then copy out the flagged set: one record per racy
 * key, sorted by (space, region, block if LDS, index), unique (races are
 * reported once per unique address, Sec. V-C).  Writes up to cap records to
 * out (host memory owned by the caller) and the full count to *n_out.  When
 * race records are missing (the ring overflowed, or a call site reached
 * site_limit) the global-memory part of the set is completed from the sticky
 * race states in shadow memory (those records carry HR_RACE_SCANNED).
 * Returns the warning bits, HR_E_INVAL (c or n_out NULL, or cap too small:
 * *n_out then holds the count), or HR_E_HIP.  The ring is not cleared (see
 * hr_reset). */
hr_status hr_report(hr_ctx c, hr_race* out, size_t cap, size_t* n_out, void* stream);

/* Synchronise `stream` and read the checked-access counter (only counts when
 * the context was created with HR_CFG_COUNT_CHECKS). */
hr_status hr_check_count(hr_ctx c, uint64_t* out, void* stream);

/* One checked access as a hook saw it (HR_CFG_ACCESS_LOG), 32 bytes: the
 * inputs of the per-access update of Algorithm 1 (Sec. IV-B: the address,
 * the access kind, the thread and its barrier clocks) plus the launch. */
typedef struct {
    uint64_t index;     /* element index (global) or LDS word */
    uint32_t region;    /* region id (global) or LDS array id */
    uint32_t block;     /* the accessing logical block (owner of an LDS word) */
    uint32_t launch;    /* launch sequence number within the job */
    uint16_t thread;    /* thread within its block */
    uint8_t space;      /* hr_space */
    uint8_t kind;       /* hr_kind */
    uint8_t bc, wc;     /* block and wave clocks */
    uint16_t site;      /* call-site id */
    uint32_t tc;        /* tile clock (a context with HR_CFG_NESTED_TILES), else 0 */
} hr_access_rec;

/* Synchronise `stream` and copy the access log of a context created with
 * HR_CFG_ACCESS_LOG into out (host memory, cap records): every access the
 * hooks checked since the context was created or last reset, in no
 * particular order.  *n_out receives the number of records held
 * (min(accesses, log_capacity)).  Returns HR_W_LOG_TRUNCATED when accesses
 * were dropped, HR_E_INVAL (c or n_out NULL, no log, or cap below *n_out),
 * HR_E_HIP.  The log is cleared by hr_reset. */
hr_status hr_access_log(hr_ctx c, hr_access_rec* out, size_t cap, size_t* n_out, void* stream);

/* Host evaluation of the device transition function, for verification of
 * the state machine; not used by the checking path.  space: hr_space; old:
 * shadow word (low 32 bits for LDS); kind: hr_kind; the identity is the
 * access's launch, block, thread-in-block and block/wave clocks; wave_bits
 * as in hr_config (6: waves, s < 6: tiles of 2^s lanes; wc counts the
 * group's barriers).  Writes the new shadow word. */
hr_status hr_fsm_step(uint32_t space, uint64_t old, uint32_t kind, uint32_t launch,
                      uint32_t block, uint32_t thread, uint32_t bc, uint32_t wc,
                      uint32_t wave_bits, uint64_t* new_out);

/* The same transition of a global word through the flat table that a
 * context made with HR_CFG_FSM_TABLE uses (for verification: it must equal
 * hr_fsm_step on every input).  Arguments as hr_fsm_step, global words only
 * (space must be HR_GLOBAL). */
hr_status hr_fsm_step_table(uint32_t space, uint64_t old, uint32_t kind, uint32_t launch,
                            uint32_t block, uint32_t thread, uint32_t bc, uint32_t wc,
                            uint32_t wave_bits, uint64_t* new_out);

/* Host evaluation of the device merge of two global shadow words (the summary
 * of the union of their access sets; x of the current launch), used when an
 * exchange overwrote a concurrent update; for verification only.  wave_bits
 * as in hr_fsm_step. */
hr_status hr_fsm_merge(uint64_t x, uint64_t y, uint32_t wave_bits, uint64_t* out);

/* Host evaluation of the transition of the nested-tile machine (contexts
 * made with HR_CFG_NESTED_TILES: tiles of 2^tile_bits lanes, tile_bits 1..5,
 * nested in the waves, each with its own barrier and tile clock tc), for
 * verification only.  space: hr_space; old: shadow word (low 32 bits for
 * LDS); the identity is the access's launch, block (< 2^20), thread (<
 * 1024) and block, wave and tile clocks (< 32, 16 and 16).  Errors:
 * HR_E_INVAL (null out, kind > 2, an identity field out of range). */
hr_status hr_fsm_step_nested(uint32_t space, uint64_t old, uint32_t kind, uint32_t launch,
                             uint32_t block, uint32_t thread, uint32_t bc, uint32_t wc,
                             uint32_t tc, uint32_t tile_bits, uint64_t* new_out);

/* Host evaluation of the nested-tile machine's merge of two global words
 * (as hr_fsm_merge), for verification only. */
hr_status hr_fsm_merge_nested(uint64_t x, uint64_t y, uint32_t tile_bits, uint64_t* out);

/* Decode a shadow summary word of `space` (for instance the `before` and
 * `with` fields of a race record) of a context with the given wave_bits: the
 * `wave` and `wc` fields then name the synchronization group (wave or tile)
 * and its clock.  Errors: HR_E_INVAL (null out, unknown space or state tag,
 * wave_bits outside 1..6). */
hr_status hr_describe(uint32_t space, uint64_t word, uint32_t wave_bits, hr_summary* out);

/* Decode a shadow summary word of `space` of a context with
 * HR_CFG_NESTED_TILES and tiles of 2^tile_bits lanes (its wave_bits): the
 * `before` and `with` fields of that context's race records use this layout
 * (paper Sec. III-A's summaries, with the tile level of the nested machine
 * added below the wave).  Errors: HR_E_INVAL (null out, unknown space or
 * state tag, tile_bits outside 1..5). */
hr_status hr_describe_nested(uint32_t space, uint64_t word, uint32_t tile_bits,
                             hr_summary_nested* out);

/* Host evaluation of the device transition on a 4-byte global word
 * (HR_CFG_WORD4) whose field widths are wc_bits, bc_bits and thread_bits
 * (as in hr_config, 0 for the defaults), for verification only.  The block
 * and thread are folded to the word's fields as on the device.  Errors:
 * HR_E_INVAL (null out, kind > 2, widths out of range, bc or wc beyond its
 * field). */
hr_status hr_fsm_step_word4(uint32_t old, uint32_t kind, uint32_t block, uint32_t thread,
                            uint32_t bc, uint32_t wc, uint32_t wave_bits, uint32_t wc_bits,
                            uint32_t bc_bits, uint32_t thread_bits, uint32_t* new_out);

/* The 8-byte global word holding the same summary as a 4-byte one (launch
 * 0), for hr_describe.  Widths as in hr_fsm_step_word4.  Errors: HR_E_INVAL
 * (null out, widths out of range, a state number above 20). */
hr_status hr_word4_widen(uint32_t word, uint32_t wc_bits, uint32_t bc_bits, uint32_t thread_bits,
                         uint64_t* out);

/* ----------------------------------------------------------------------
 * Instrumented workloads.  Each *_check entry launches one instrumented
 * kernel on `stream` (the caller calls hr_kernel_end after it); each *_plain
 * entry launches the same kernel without hooks.  Data pointers are device
 * pointers; region ids come from hr_shadow_alloc on those buffers.
 * Errors: HR_E_INVAL (bad sizes, regions too small), HR_E_HIP.
 * ---------------------------------------------------------------------- */

/* Call-site ids carried by the workloads' race records. */
enum {
    /* reduction */
    HR_SITE_REDUCE_LOAD = 1,        /* global read of the input */
    HR_SITE_REDUCE_STAGE = 2,       /* LDS write of the loaded value */
    HR_SITE_REDUCE_LEFT = 3,        /* LDS read of a[t] in a halving step */
    HR_SITE_REDUCE_RIGHT = 4,       /* LDS read of a[t + h] */
    HR_SITE_REDUCE_SUM = 5,         /* LDS write of a[t] */
    HR_SITE_REDUCE_TOTAL = 6,       /* LDS read of a[0] after the steps */
    HR_SITE_REDUCE_OUT = 7,         /* global write of the output */
    /* stencil */
    HR_SITE_JACOBI_CENTRE = 16,     /* global read of the thread's own cell */
    HR_SITE_JACOBI_HALO = 17,       /* global read of a halo cell */
    HR_SITE_JACOBI_STAGE = 18,      /* LDS write into the tile */
    HR_SITE_JACOBI_TILE = 19,       /* LDS read of the centre or a neighbour */
    HR_SITE_JACOBI_OUT = 20,        /* global write of the thread's own cell */
    HR_SITE_JACOBI_SEED = 21,       /* seeded global write of a neighbour's cell */
    /* label propagation */
    HR_SITE_LP_OWN = 32,            /* atomic load of the vertex's own label */
    HR_SITE_LP_CSR = 33,            /* read of row_ptr or col (when monitored) */
    HR_SITE_LP_MIN = 34,            /* atomic min into a neighbour's label */
    HR_SITE_LP_SEED_READ = 35,      /* seeded plain read of a neighbour's label */
    HR_SITE_LP_SEED_WRITE = 36      /* seeded plain write of a neighbour's label */
    /* access programs: site = phase + 1 */
};

/* LDS tree reduction: each of `blocks` blocks of `threads` threads (a
 * multiple of 64, <= 1024) sums in_dev[b*n .. b*n+n) (int32; n a power of
 * two, 2 <= n <= 2*threads) in LDS over log2(n) halving steps with a block
 * barrier after each (and one after the loads when n != 2*threads); every
 * thread then writes its block's sum to out_dev[b*threads + t].  drop
 * names a step whose barrier is removed (a seeded race); a value outside
 * 0..log2(n)-1 keeps all barriers.  LDS array id 0.  The paper-sized case
 * is n = 512, threads = 256, blocks = 1.  HR_E_INVAL also for a context
 * with HR_CFG_NESTED_TILES or HR_CFG_FSM_TABLE. */
hr_status hr_reduce_check(hr_ctx c, uint32_t r_in, uint32_t r_out, const int32_t* in_dev,
                          int32_t* out_dev, uint32_t n, uint32_t threads, uint32_t blocks,
                          int32_t drop, void* stream);
hr_status hr_reduce_plain(const int32_t* in_dev, int32_t* out_dev, uint32_t n, uint32_t threads,
                          uint32_t blocks, int32_t drop, void* stream);

/* One 5-point Jacobi sweep u_new = 0.2 (c + n + s + w + e) over an ny x nx
 * fp32 grid (row-major), 16x16-thread blocks staging an 18x18 LDS tile (LDS
 * array id 0; corners unused); neighbours outside the grid read the centre
 * value.  seed_dev: NULL or int32 per block (row-major block order): -1, or
 * side << 8 | offset, in which case that block's edge thread next to halo
 * cell `offset` on `side` (0 N, 1 S, 2 W, 3 E) also writes that
 * neighbour-owned cell of u_new (a seeded cross-block race).  A context
 * with HR_CFG_FSM_TABLE runs the table kernel, on row-major maps only
 * (HR_E_INVAL for tiled regions); one with HR_CFG_NESTED_TILES is
 * rejected (HR_E_INVAL). */
hr_status hr_jacobi_check(hr_ctx c, uint32_t r_old, uint32_t r_new, const float* u_old_dev,
                          float* u_new_dev, uint32_t ny, uint32_t nx, const int32_t* seed_dev,
                          void* stream);
hr_status hr_jacobi_plain(const float* u_old_dev, float* u_new_dev, uint32_t ny, uint32_t nx,
                          const int32_t* seed_dev, void* stream);

/* One label-propagation sweep over a CSR graph (row_ptr_dev[n+1],
 * col_dev[m], int32), one thread per vertex v in blocks of tpb threads:
 * l = atomic load of label[v]; for every edge (v, u): atomic min of l into
 * label[u], or, where mask_dev[e] != 0, a plain read and plain write of
 * label[u] (a seeded race).  r_row_ptr / r_col: region ids to also monitor
 * the CSR reads, or UINT32_MAX.  All pointers must be non-NULL (a graph
 * without edges still passes some col and mask buffer), else HR_E_INVAL;
 * row_ptr_dev[n] must not exceed the length of col_dev and mask_dev, which
 * is not checked (it lies in device memory).  Limits: 1 <= tpb <= 1024,
 * ceil(n / tpb) < 2^22 blocks.  HR_E_INVAL also for a context with
 * HR_CFG_NESTED_TILES or HR_CFG_FSM_TABLE. */
hr_status hr_labelprop_check(hr_ctx c, uint32_t r_label, uint32_t r_row_ptr, uint32_t r_col,
                             int32_t* label_dev, const int32_t* row_ptr_dev,
                             const int32_t* col_dev, const uint8_t* mask_dev, uint32_t n,
                             uint32_t tpb, void* stream);
hr_status hr_labelprop_plain(int32_t* label_dev, const int32_t* row_ptr_dev,
                             const int32_t* col_dev, const uint8_t* mask_dev, uint32_t n,
                             uint32_t tpb, void* stream);

/* One launch of an access program: `blocks` blocks of `threads` threads run
 * `phases` phases; in phase p thread t of logical block b performs the
 * operations ops_dev[op_off_dev[i] .. op_off_dev[i+1]) with
 * i = (p * blocks + b) * threads + t, then the phase ends with nothing
 * (scope 0), a wave barrier in waves (tiles, when the context's wave_bits
 * is below 6) whose bit is set in wave_mask_dev[p] (scope 1; groups past the
 * 64th never synchronize), a block barrier (scope 2), or, in a context with
 * HR_CFG_NESTED_TILES, a tile barrier in the tiles whose bit is set (scope
 * 3; scope 1 then orders whole waves).  Operation word: bits 0..23 index,
 * 24..26 program region (global: regions_host[region] is the context region;
 * LDS: array 0 of lds_words int32), 27..28 hr_kind, or 3 for an operation
 * that switches the thread's checking off (bit 0 clear) or on (bit 0 set)
 * with hr_thread_enable, 29 space.  Reads load,
 * writes store, atomics add 1.  block_map_dev: NULL or a permutation giving
 * the logical block of each hardware block.  n_ops / n_op_off bound the
 * arrays; out-of-range operations are skipped and reported as
 * HR_W_OUT_OF_RANGE.  Limits: threads <= 1024, lds_words <= 8192. */
hr_status hr_program_check(hr_ctx c, const uint32_t* regions_host, uint32_t n_regions,
                           uint32_t blocks, uint32_t threads, uint32_t phases,
                           const uint8_t* scope_dev, const uint64_t* wave_mask_dev,
                           const int32_t* op_off_dev, size_t n_op_off, const uint32_t* ops_dev,
                           size_t n_ops, const uint32_t* block_map_dev, uint32_t lds_words,
                           void* stream);

/* ----------------------------------------------------------------------
 * Batched checking: many independent checked jobs in one persistent launch.
 * ---------------------------------------------------------------------- */

#define HR_PAT_REDUCE 0u      /* hr_reduce_check's kernel, phases = 1 */
#define HR_PAT_JACOBI 1u      /* hr_jacobi_check's kernel, ping-pong over phases */
#define HR_PAT_LABELPROP 2u   /* hr_labelprop_check's kernel (CSR not monitored) */

/* One checked job.  A phase is one launch of the job's kernel.
 *  reduce:    n = words per block, threads, blocks, drop; data[0] = in,
 *             data[1] = out.
 *  jacobi:    n = columns (nx), ny = rows; data[0] = u0, data[1] = u1
 *             (phase p reads u[p%2] and writes u[(p+1)%2]), data[2] = NULL
 *             or the per-block seed table; blocks and threads are derived.
 *  labelprop: n = vertices, threads = block size; data[0] = label,
 *             data[1] = row_ptr, data[2] = col, data[3] = seeded-edge mask;
 *             blocks is derived.
 * region[] is written by hr_batch_create: the context regions holding the
 * job's shadow (reduce in/out, jacobi u0/u1, labelprop label / UINT32_MAX).
 * LDS race records of a batched job carry region[0] as their array id. */
typedef struct {
    uint32_t pattern;
    uint32_t blocks, threads, phases;   /* phases: 1..512 */
    uint32_t n, ny;
    int32_t drop;
    uint32_t region[2];
    uint32_t pad;
    const void* data[4];
} hr_instance;

typedef struct hr_batch_s* hr_batch;

typedef struct {
    uint32_t workers;     /* resident worker blocks; 0 or too many: all that fit */
    uint32_t order;       /* 0: phase-major queue; 1: phase-major, largest jobs first */
    uint32_t spin_limit;  /* wait rounds before an item is skipped; 0: 2^24 */
    uint32_t variant;     /* 0: one worker per compute unit, 128 registers per lane;
                             1: two workers per compute unit, 64 registers */
    uint32_t coalesce;    /* wave grouping of the lanes of one hook instruction
                             that hit the same shadow word, at data-dependent
                             sites: 0 the context's setting, 1 off, or the
                             coalescing width (a power of two, 2..64: lanes
                             group within aligned segments of that many); the
                             result is the same either way */
    uint32_t tile;        /* shadow map of the stencil jobs' grids: tw | th << 4
                             (tiles of 2^tw columns by 2^th rows, each side at
                             most 2^HR_TILE_LOG2_MAX; 0: row-major), as
                             hr_shadow_alloc_2d; it stays for later runs and
                             reports.  The result is the same for every map. */
} hr_batch_tuning;

/* Prepare a batch: allocate one shadow arena for every job (counted against
 * the context's shadow budget), register its regions in the context, build
 * the work queues (instance, phase, block) and upload the job table.  inst
 * stays owned by the caller; region[] is filled in.  Errors: HR_E_INVAL (a
 * job's shape, a context with HR_CFG_WORD4, HR_CFG_NESTED_TILES or
 * HR_CFG_FSM_TABLE), HR_E_NOMEM, HR_E_HIP. */
hr_status hr_batch_create(hr_ctx c, hr_instance* inst, uint32_t n_inst, hr_batch* out);

/* Run every job of the batch to completion in one persistent launch of
 * 1024-thread worker blocks on `stream`: worker blocks claim items in queue
 * order; an item of phase p waits until every block of phase p-1 of its job
 * has finished, and the job's shadow words carry p as their launch epoch.
 * Clears the batch's shadow and phase counters first.  Races go to the
 * context's ring (read them with hr_report).  Asynchronous. */
hr_status hr_batch_run(hr_batch b, const hr_batch_tuning* tune, void* stream);

/* Number of worker blocks of kernel `variant` that fit on the device, and of
 * work items. */
hr_status hr_batch_info(hr_batch b, uint32_t variant, uint32_t* max_workers, uint64_t* items);

/* Free the batch's queues and shadow arena (its regions become invalid).
 * Synchronises the context's stream. */
hr_status hr_batch_destroy(hr_batch b);

/* The serial path for one job: create a context with cfg, allocate its
 * shadow, launch each phase with the job's *_check kernel and a launch
 * boundary, report into out (as hr_report; region ids 0 and 1), and free
 * everything.  Synchronous. */
hr_status hr_job_run(const hr_instance* inst, const hr_config* cfg, hr_race* out, size_t cap,
                     size_t* n_out, void* stream);

/* Size of the library's static scratch array and its parts (see
 * hr_job_run_static). */
#define HR_STATIC_SCRATCH_BYTES (64u << 20)
#define HR_STATIC_RING_RECORDS 16384u
#define HR_STATIC_SHADOW_WORDS 8289280u   /* 8-byte words after counters and ring */

/* hr_job_run for callers that cannot allocate device memory (code that must
 * not call hipMalloc, tight serving loops, harnesses that forbid
 * allocation): the same job, launches and report, but the counters, the
 * report ring (at most HR_STATIC_RING_RECORDS records; a larger
 * cfg->ring_capacity is capped) and the shadow words live in one static
 * device array of HR_STATIC_SCRATCH_BYTES that the library holds on each
 * device it runs on until the process ends.  The call allocates nothing, on
 * the device or through any allocating library routine; it clears the parts
 * of the array it uses before the first launch, so nothing of an earlier
 * call is seen.  Calls of one process are serialised by a lock (each
 * shares that device's array); two library instances that drive the same
 * array at once would race.  Synchronous, on `stream`.  out (host memory,
 * cap records) also serves as the working buffer of the report: cap must
 * hold the raw records (ring records before deduplication, plus every
 * global race word when records were dropped), else HR_E_INVAL with *n_out
 * = that number; on success *n_out is the number of unique records, sorted
 * as by hr_report.  Returns the warning bits as hr_report does.
 * Errors: HR_E_INVAL (a job's shape, cfg out of range or with
 * HR_CFG_WORD4, cap too small), HR_E_NOMEM (the job's two buffers need more
 * than HR_STATIC_SHADOW_WORDS shadow words), HR_E_HIP. */
hr_status hr_job_run_static(const hr_instance* inst, const hr_config* cfg, hr_race* out,
                            size_t cap, size_t* n_out, void* stream);

/* ----------------------------------------------------------------------
 * Serving: a stream of jobs checked with continuous batching.
 *
 * A job's launches run one after another (Sec. II-B: a kernel boundary
 * orders everything before it), so a device iteration may run the next
 * phase of every resident job side by side.  Jobs are admitted in arrival
 * order, while a job slot, shadow memory under the budget and room under
 * the item cap are free; a job's shadow words stay resident until its last
 * phase has been reported.  Jobs run in four lanes by class (short jobs;
 * label propagation under 64 items per phase; label propagation of 64 items
 * or more; other jobs of more than 1024 items per phase); each lane runs its
 * own iterations, and the lanes' iterations overlap on the device.  The
 * large-job lane runs one job at a time, in admission order; a stencil job
 * there runs large_burst phases per iteration, as launches of the kernel
 * hr_jacobi_check runs. 
 * ---------------------------------------------------------------------- */

typedef struct {
    double arrival_s;   /* in: arrival time, seconds after the call starts;
                           non-decreasing over the job list */
    double admit_s;     /* out: when the job was admitted (its shadow placed) */
    double finish_s;    /* out: when its last phase was reported */
    uint32_t flagged;   /* out: distinct flagged locations of the job */
    int32_t status;     /* out: HR_W_* bits of the iterations the job ran in
                           (serial path: the job's hr_job_run status) */
} hr_serve_job;

typedef struct {
    uint64_t shadow_budget;  /* bytes of shadow resident at once; 0: 64 GiB */
    uint32_t max_slots;      /* jobs resident at once, < 2^20; 0: 1024 */
    uint32_t serial;         /* nonzero: replay the arrivals one job at a time
                                through hr_job_run (the plain path) */
    uint32_t max_items;      /* work items (1024-thread blocks) of the resident
                                jobs' phases in one iteration, at most
                                HR_SERVE_MAX_ITEMS; 0: HR_SERVE_MAX_ITEMS */
    uint32_t large_burst;    /* phases of a large stencil job that one iteration
                                of the large-job lane runs; 0: all remaining */
    uint32_t lane_burst;     /* phases one iteration of the short-job lane
                                runs: the next lane_burst phases of its
                                resident jobs, as launches back to back; 0: 2,
                                at most 64 */
    uint32_t pad;
} hr_serve_config;

/* One iteration is one launch of 1024-thread blocks, whose grid may not
 * exceed 2^32 - 1 threads. */
#define HR_SERVE_MAX_ITEMS ((1u << 22) - 1u)

/* Check n_jobs jobs (hr_instance as for hr_batch_create; region[] unused)
 * arriving at times[j].arrival_s, on the context's device and `stream`, and
 * wait for all of them.  The call paces itself by the arrival times (it
 * sleeps while nothing is resident).  Race records of job j carry region id
 * 2j (its first buffer, and its LDS arrays) or 2j+1 (its second buffer); out
 * receives every job's deduplicated records, sorted by (region, space,
 * block if LDS, index); *n_out is their number.  The first lane runs on
 * `stream` with the context's ring and counters; the call creates three
 * non-blocking streams (default priority) and their rings for the other
 * lanes, and frees them before it returns.  The context's regions are not
 * touched.
 * Errors: HR_E_INVAL (a context with HR_CFG_WORD4, HR_CFG_NESTED_TILES or
 * HR_CFG_FSM_TABLE, a job's shape, unsorted arrivals, max_items above
 * HR_SERVE_MAX_ITEMS, a job with more items per phase than max_items,
 * lane_burst above 64, cap too small: then *n_out holds the number needed),
 * HR_E_NOMEM (a job larger than the budget, or the device allocation
 * failed), HR_E_HIP. */
hr_status hr_serve(hr_ctx c, const hr_instance* jobs, hr_serve_job* times, uint32_t n_jobs,
                   const hr_serve_config* cfg, hr_race* out, size_t cap, size_t* n_out,
                   void* stream);

/* ----------------------------------------------------------------------
 * Device microbenchmarks: the roofline denominators of the checking path
 * (its cost is HBM traffic of shadow words and agent-scope atomics).
 * ---------------------------------------------------------------------- */

/* Copy `bytes` (a multiple of 16) from src_dev to dst_dev with 16-byte
 * vector loads and stores: streaming HBM bandwidth, and the calibration
 * kernel for the HBM byte counters. */
hr_status hr_peak_copy(const void* src_dev, void* dst_dev, size_t bytes, void* stream);

/* One agent-scope 64-bit atomic per word of words_dev[n]: op 0 is a
 * compare-and-swap from `round` to round+1, op 1 an exchange writing round+1
 * (the two forms the checking path uses).  Every word must hold `round`;
 * scatter 1 permutes words within 64 KiB windows (n should be a multiple of
 * 8192) so the lanes of a wave hit different cache lines; scatter 2 (n a
 * power of two) spreads consecutive operations over the whole array.  Operations that
 * found another value are added to *fails_dev.  blocks: blocks of 256
 * threads, each thread taking every (blocks * 256)-th word; 0 gives one word
 * per thread (at most 65536 blocks).  Fewer, longer-running blocks keep more
 * operations in flight per wave, so a peak is the best over a few. */
hr_status hr_peak_atomic(uint64_t* words_dev, size_t n, uint32_t op, uint32_t round,
                         uint32_t scatter, uint32_t* fails_dev, uint32_t blocks, void* stream);

/* LDS 32-bit compare-and-swap throughput: `blocks` blocks of 1024 threads,
 * each thread taking its own LDS word through `iters` successful
 * compare-and-swaps (op 0), or each time a load then a compare-and-swap from
 * the loaded value (op 1, the LDS hook's pattern): blocks * 1024 * iters
 * operations.  A failed operation is added to *fails_dev. */
hr_status hr_peak_lds(uint32_t blocks, uint32_t iters, uint32_t op, uint32_t* fails_dev,
                      void* stream);

/* One agent-scope (coherent) 64-bit atomic load per word of words_dev[n],
 * same index patterns as hr_peak_atomic; sink_dev receives nothing unless an
 * improbable value appears (it keeps the loads from being removed). */
hr_status hr_peak_load(const uint64_t* words_dev, size_t n, uint32_t scatter, uint64_t* sink_dev,
                       void* stream);

#ifdef __cplusplus
}
#endif

#endif /* HR_H */
