// Per-location race-check state machine and its shadow-word encodings.
//
// The paper (Sec. III, "Design of HiRace") summarises the whole access
// history of one memory location by the hierarchical scope shared by its
// accessors plus the last accessor's identity and barrier clocks, packed in a
// constant-size shadow word and advanced by an atomic compare-and-swap
// (Sec. IV-B, Algorithm 1: unpack, compare thread ids, check sync, look up
// the transition, pack).  Its full 25-state machine is not published; the
// machine below is this library's own, built on the same idea and exact for
// launch, block-barrier and wave-barrier happens-before.
//
// Access classes: R = plain reads only, A = atomics only, X = a write, or
// reads and atomics together.  Encoded as 2-bit masks R=1, A=2, X=3 so that
// the join of two classes is their OR, and class c conflicts with access
// class k exactly when (c | k) == 3 (two reads never conflict, two atomics
// never conflict, everything else does; Sec. II-A and Sec. III-B).
//
// States (tag + classes), relative to the current launch:
//   INIT               never accessed (all-zero word)
//   RACE               a race has been seen (sticky)
//   MB(k)              accesses from >= 2 blocks, all of class k in {R, A}
//   MW(cL, k)          one block; in its latest block epoch >= 2 waves, all
//                      of class k; cL = class of the block's whole launch
//   MT(cL, cB, k)      one block, one wave in the latest block epoch (class
//                      cB); >= 2 threads in that wave's latest wave epoch,
//                      all of class k
//   ST(cL, cB, cW)     as MT but one thread in the latest wave epoch, of
//                      class cW
// with cW <= cB <= cL in the class order.  Homogeneous multi-accessor summaries
// are exact because any two of their accesses from different threads are
// unordered, so they hold a concurrent access of class k from another
// accessor for every later access in the same scope and epoch.
//
// A state keeps only the identity fields it needs (launch; + block, block
// clock; + wave, wave clock; + thread), which makes the encoding canonical:
// an access that changes nothing produces exactly the old word, and the hook
// skips its compare-and-swap.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#define HR_HD __host__ __device__ __forceinline__
#else
#define HR_HD inline
#endif

namespace hr {

enum : uint32_t { CL_R = 1u, CL_A = 2u, CL_X = 3u };
enum : uint32_t { T_INIT = 0u, T_RACE = 1u, T_MB = 2u, T_MW = 3u, T_MT = 4u, T_ST = 5u };

// Access kinds of the C ABI (plain read, plain write, atomic) -> class.
HR_HD constexpr uint32_t kind_class(uint32_t kind)
{
    return kind == 0u ? CL_R : (kind == 2u ? CL_A : CL_X);
}
HR_HD constexpr bool conflicts(uint32_t cls, uint32_t k) { return (cls | k) == CL_X; }

// ---------------------------------------------------------------------------
// Global-memory shadow word, 64 bits, least significant first:
//   tag 3 | cW 2 | cB 2 | cL 2 | wc 6 | bc 8 | thread 10 | block 22 | launch 9
// The wave of a thread is the top 4 bits of its 10-bit thread index.  A
// context may instead synchronize tiles of 2^s lanes (s < 6): then the
// "wave" level of the machine is the tile (the top 10 - s bits of the thread
// index), wave barriers are tile barriers, and wc counts them.  The split is
// passed to step and merge as the mask of the group bits (group_mask(s)).
// ---------------------------------------------------------------------------
namespace g {
constexpr uint32_t TAG_SH = 0, CW_SH = 3, CB_SH = 5, CL_SH = 7, WC_SH = 9, BC_SH = 15,
                   TH_SH = 23, BL_SH = 33, LA_SH = 55;
constexpr uint64_t TAG_M = 7ull << TAG_SH;
constexpr uint64_t CW_M = 3ull << CW_SH, CB_M = 3ull << CB_SH, CL_M = 3ull << CL_SH;
constexpr uint64_t WC_M = 63ull << WC_SH;
constexpr uint64_t BC_M = 255ull << BC_SH;
constexpr uint64_t TH_M = 1023ull << TH_SH;          // thread within the block
constexpr uint64_t LANE_M = 63ull << TH_SH;           // thread within its wave
constexpr uint64_t WAVE_M = 15ull << (TH_SH + 6);     // wave within the block

// Mask of the thread bits naming the synchronization group: the wave (s =
// 6) or a tile of 2^s lanes.
HR_HD constexpr uint64_t group_mask(uint32_t s)
{
    return (uint64_t)((1023u >> s) << s) << TH_SH;
}
constexpr uint64_t BL_M = ((1ull << 22) - 1) << BL_SH;
constexpr uint64_t LA_M = 511ull << LA_SH;
constexpr uint32_t BLOCK_LIMIT = 1u << 22;
constexpr uint32_t LAUNCH_BITS = 9;

// Identity fields of the accessing thread, packed in place.
HR_HD constexpr uint64_t pack_id(uint32_t launch, uint32_t block, uint32_t thread, uint32_t bc,
                                 uint32_t wc)
{
    return ((uint64_t)(launch & 511u) << LA_SH) | ((uint64_t)(block & (BLOCK_LIMIT - 1)) << BL_SH) |
           ((uint64_t)(thread & 1023u) << TH_SH) | ((uint64_t)(bc & 255u) << BC_SH) |
           ((uint64_t)(wc & 63u) << WC_SH);
}

HR_HD constexpr uint64_t mk(uint32_t tag, uint32_t cl, uint32_t cb, uint32_t cw)
{
    return ((uint64_t)tag << TAG_SH) | ((uint64_t)cl << CL_SH) | ((uint64_t)cb << CB_SH) |
           ((uint64_t)cw << CW_SH);
}

// One transition: old shadow word, identity of the access, class k of the
// access, mask of the group bits of the thread index.
HR_HD constexpr uint64_t step(uint64_t old, uint64_t id, uint32_t k, uint64_t wm = WAVE_M)
{
    const uint32_t tag = (uint32_t)(old & TAG_M);
    if (tag == T_RACE) return old;
    const uint64_t d = old ^ id;
    const uint32_t cl = (uint32_t)(old >> CL_SH) & 3u;
    const uint32_t cb = (uint32_t)(old >> CB_SH) & 3u;
    const uint32_t cw = (uint32_t)(old >> CW_SH) & 3u;
    const uint64_t race = T_RACE;
    const uint64_t lm = TH_M & ~wm;
    const uint64_t keep_t = LA_M | BL_M | BC_M | TH_M | WC_M;   // ST
    const uint64_t keep_w = LA_M | BL_M | BC_M | wm | WC_M;     // MT
    const uint64_t keep_b = LA_M | BL_M | BC_M;                           // MW
    // First access of this launch: everything earlier is ordered before it.
    if (tag == T_INIT || (d & LA_M)) return mk(T_ST, k, k, k) | (id & keep_t);
    // >= 2 blocks: every access meets a concurrent one of class cb.
    if (tag == T_MB) return conflicts(cb, k) ? race : old;
    // Another block: concurrent with everything the stored block did.
    if (d & BL_M) return conflicts(cl, k) ? race : (mk(T_MB, 0, k, 0) | (id & LA_M));
    // Same block, later block epoch: ordered after the stored history.
    if (d & BC_M) return mk(T_ST, cl | k, k, k) | (id & keep_t);
    // Same block epoch with >= 2 waves.
    if (tag == T_MW) return conflicts(cb, k) ? race : old;
    // Another wave in the same block epoch.
    if (d & wm) return conflicts(cb, k) ? race : (mk(T_MW, cl, k, 0) | (id & keep_b));
    // Same wave, later wave epoch.
    if (d & WC_M) return mk(T_ST, cl | k, cb | k, k) | (id & keep_t);
    // Same wave epoch with >= 2 threads.
    if (tag == T_MT) return conflicts(cw, k) ? race : old;
    // Another thread of the same wave epoch.
    if (d & lm) return conflicts(cw, k) ? race : (mk(T_MT, cl, cb, k) | (id & keep_w));
    // Same thread.
    return mk(T_ST, cl | k, cb | k, cw | k) | (id & keep_t);
}

// ---------------------------------------------------------------------------
// The same transition as a flat table (the paper's encoding of its machine,
// Sec. IV-B: an array indexed by the old state and the transition labels).
// The labels are the relation of the access to the stored history -- 0 new
// launch (or an initial word), 1 other block, 2 later block epoch, 3 other
// wave, 4 later wave epoch, 5 other thread, 6 same thread, decided from the
// XOR of the two words in that order -- and the access class.  The index
// concatenates the old tag (3 bits), the relation (3 bits), the old word's
// class fields cW, cB, cL (its bits 3..8) and the access class; the entry
// is the new word's low 9 bits (tag and classes), or TAB_SAME for an
// unchanged word.  The identity fields the new state keeps come from the
// access (ST: thread; MT: group; MW: block; MB: launch; RACE: none).  The
// table is built at compile time from step() itself, so both encodings are
// one machine; which one runs faster is a matter of measurement.
// ---------------------------------------------------------------------------
constexpr uint32_t TAB_SIZE = 64u << 8;   // every 3-bit tag (words of other tags are
                                          // not made by the machine, but any word reads
                                          // an entry inside the table)
constexpr uint16_t TAB_SAME = 0x8000u;

struct step_table {
    uint16_t e[TAB_SIZE];
};

HR_HD constexpr uint32_t relation(uint64_t old, uint64_t id, uint64_t wm)
{
    const uint64_t d = old ^ id;
    const uint32_t tag = (uint32_t)(old & TAG_M);
    return (tag == T_INIT || (d & LA_M)) ? 0u
           : (d & BL_M)                  ? 1u
           : (d & BC_M)                  ? 2u
           : (d & wm)                    ? 3u
           : (d & WC_M)                  ? 4u
           : (d & (TH_M & ~wm))          ? 5u
                                         : 6u;
}

HR_HD constexpr uint32_t tab_index(uint64_t old, uint32_t rel, uint32_t k)
{
    return ((((uint32_t)(old & TAG_M) << 3) | rel) << 8) | ((uint32_t)(old >> CW_SH) & 63u) << 2 | k;
}

// Identity fields a word of tag `tag` keeps.
HR_HD constexpr uint64_t keep_of(uint32_t tag, uint64_t wm)
{
    return tag == T_ST   ? (LA_M | BL_M | BC_M | TH_M | WC_M)
           : tag == T_MT ? (LA_M | BL_M | BC_M | wm | WC_M)
           : tag == T_MW ? (LA_M | BL_M | BC_M)
           : tag == T_MB ? LA_M
                         : 0ull;
}

// A stored word and an access in relation `rel` to it: identity fields that
// differ from the word's in exactly the field the relation names.
HR_HD constexpr uint64_t rel_id(uint32_t rel)
{
    return rel == 0u   ? pack_id(2, 5, 67, 3, 2)
           : rel == 1u ? pack_id(1, 6, 67, 3, 2)
           : rel == 2u ? pack_id(1, 5, 67, 4, 2)
           : rel == 3u ? pack_id(1, 5, 131, 3, 2)
           : rel == 4u ? pack_id(1, 5, 67, 3, 3)
           : rel == 5u ? pack_id(1, 5, 68, 3, 2)
                       : pack_id(1, 5, 67, 3, 2);
}

constexpr step_table make_step_table()
{
    step_table t{};
    for (uint32_t tag = 0; tag < 8; ++tag)
        for (uint32_t rel = 0; rel < 8; ++rel)
            for (uint32_t c = 0; c < 64; ++c)
                for (uint32_t k = 0; k < 4; ++k) {
                    const uint32_t i = (((tag << 3) | rel) << 8) | (c << 2) | k;
                    if (rel > 6 || k == 0) {
                        t.e[i] = TAB_SAME;
                        continue;
                    }
                    const uint64_t old = (uint64_t)tag | ((uint64_t)c << CW_SH) |
                                         (tag == T_INIT ? 0ull : pack_id(1, 5, 67, 3, 2));
                    const uint64_t nw = step(old, rel_id(rel), k, WAVE_M);
                    t.e[i] = nw == old ? TAB_SAME : (uint16_t)(nw & 511u);
                }
    return t;
}

// On the representatives the table was built from, table entry plus kept
// identity fields rebuild step()'s word (checked at compile time where the
// device table is defined).
constexpr bool step_table_consistent()
{
    const step_table t = make_step_table();
    for (uint32_t tag = 0; tag < 8; ++tag)
        for (uint32_t rel = 0; rel < 7; ++rel)
            for (uint32_t c = 0; c < 64; ++c)
                for (uint32_t k = 1; k < 4; ++k) {
                    const uint64_t old = (uint64_t)tag | ((uint64_t)c << CW_SH) |
                                         (tag == T_INIT ? 0ull : pack_id(1, 5, 67, 3, 2));
                    const uint64_t id = rel_id(rel);
                    if (relation(old, id, WAVE_M) != rel && tag != T_INIT) return false;
                    const uint64_t nw = step(old, id, k, WAVE_M);
                    const uint16_t e = t.e[tab_index(old, relation(old, id, WAVE_M), k)];
                    const uint64_t got =
                        e == TAB_SAME ? old : ((uint64_t)e | (id & keep_of(e & 7u, WAVE_M)));
                    if (got != nw) return false;
                }
    return true;
}

// One transition through the table `tab` (make_step_table()).
HR_HD uint64_t step_tab(const uint16_t* tab, uint64_t old, uint64_t id, uint32_t k,
                        uint64_t wm = WAVE_M)
{
    if ((old & TAG_M) == T_RACE) return old;
    const uint16_t e = tab[tab_index(old, relation(old, id, wm), k)];
    if (e == TAB_SAME) return old;
    return (uint64_t)e | (id & keep_of(e & 7u, wm));
}

// Summary of the union of the access sets summarised by x and y, where x
// belongs to the current launch (an initial y, or one of another launch,
// adds nothing).  Used to fold
// back an update that a concurrent exchange overwrote.  Exact under the
// condition the hook guarantees: every access in one summary but not the
// other either comes from another block (then the union spans >= 2 blocks)
// or lies in the latest block epoch, and within one wave in the latest wave
// epoch, of both summaries, because a thread still inside its hook holds
// back its own block and wave barriers.  With accesses from >= 2 blocks
// (or waves, or threads) in the same scope and epoch, the union is free of
// races exactly when all of it has one class, R or A.
HR_HD uint64_t merge(uint64_t x, uint64_t y, uint64_t wm = WAVE_M)
{
    const uint32_t tx = (uint32_t)(x & TAG_M), ty = (uint32_t)(y & TAG_M);
    const uint64_t race = T_RACE;
    if (tx == T_RACE || ty == T_RACE) return race;
    if (ty == T_INIT || ((x ^ y) & LA_M)) return x;
    if (tx == T_INIT) return y;
    const uint32_t clx = (uint32_t)(x >> CL_SH) & 3u, cly = (uint32_t)(y >> CL_SH) & 3u;
    const uint32_t cbx = (uint32_t)(x >> CB_SH) & 3u, cby = (uint32_t)(y >> CB_SH) & 3u;
    const uint32_t cwx = (uint32_t)(x >> CW_SH) & 3u, cwy = (uint32_t)(y >> CW_SH) & 3u;
    const uint64_t d = x ^ y;
    const uint64_t la = x & LA_M;
    // >= 2 blocks: one class for everything, or a race.
    if (tx == T_MB || ty == T_MB || (d & BL_M)) {
        const uint32_t c = (tx == T_MB ? cbx : clx) | (ty == T_MB ? cby : cly);
        return c == CL_X ? race : (mk(T_MB, 0, c, 0) | la);
    }
    const uint32_t cl = clx | cly;
    // One block.  Different latest block epochs: the older summary's epoch
    // is ordered before the newer one's, which keeps its detail.  Clocks
    // never wrap (an overflow stops checking), so the larger one is newer.
    if (d & BC_M) {
        const uint64_t newer = (x & BC_M) > (y & BC_M) ? x : y;
        return (newer & ~CL_M) | ((uint64_t)cl << CL_SH);
    }
    const uint64_t keep_b = LA_M | BL_M | BC_M;
    const uint64_t keep_w = keep_b | wm | WC_M;
    // Same block epoch with >= 2 waves.
    if (tx == T_MW || ty == T_MW || (d & wm)) {
        const uint32_t c = cbx | cby;
        return c == CL_X ? race : (mk(T_MW, cl, c, 0) | (x & keep_b));
    }
    const uint32_t cb = cbx | cby;
    // One wave.  Different latest wave epochs: keep the newer detail.
    if (d & WC_M) {
        const uint64_t newer = (x & WC_M) > (y & WC_M) ? x : y;
        return (newer & ~(CL_M | CB_M)) | ((uint64_t)cl << CL_SH) | ((uint64_t)cb << CB_SH);
    }
    // Same wave epoch with >= 2 threads.
    if (tx == T_MT || ty == T_MT || (d & (TH_M & ~wm))) {
        const uint32_t c = cwx | cwy;
        return c == CL_X ? race : (mk(T_MT, cl, cb, c) | (x & keep_w));
    }
    // Same thread.
    return mk(T_ST, cl, cb, cwx | cwy) | (x & ~(TAG_M | CL_M | CB_M | CW_M));
}
}  // namespace g

// ---------------------------------------------------------------------------
// Global-memory shadow word, 32 bits (the 4-byte footprint variant):
//   state 5 | wc W | bc B | thread T | block K,   K = 27 - W - B - T.
// The 21 states reachable in the machine above (INIT, RACE, MB(k), 4 MW,
// 6 MT, 7 ST) are numbered 0..20; W, B and T are the context's clock and
// thread widths.  There is no launch field: the runtime returns every word
// to INIT at each launch boundary instead.  Widening a word gives the 64-bit
// word of the same summary (launch 0, the block as stored), so transitions
// and merges are the 64-bit ones.  Exact while a launch's block ids, thread
// indices and clocks fit their fields.  Block ids and thread indices beyond
// them are folded (taken modulo 2^K and 2^T), which makes distinct accessors
// look alike: accesses of two blocks (threads) that share a folded id are
// treated as one block's (thread's), which can hide a race but never
// creates one.
// The layout travels as one word: bc_sh | th_sh << 8 | bl_sh << 16 (the wave
// clock always starts at bit 5); 0 means the 64-bit word.
// ---------------------------------------------------------------------------
namespace c {
constexpr uint32_t STATE_BITS = 5, WC_SH = 5, N_STATES = 21;

constexpr uint32_t layout(uint32_t wc_bits, uint32_t bc_bits, uint32_t thread_bits)
{
    return (WC_SH + wc_bits) | ((WC_SH + wc_bits + bc_bits) << 8) |
           ((WC_SH + wc_bits + bc_bits + thread_bits) << 16);
}
// The default widths (wave clock 1, block clock 2, thread 8: a 16-bit block
// field), for which kernels can be compiled with the layout as a constant.
constexpr uint32_t DEFAULT_LAYOUT = layout(1, 2, 8);
HR_HD uint32_t bc_sh(uint32_t lay) { return lay & 255u; }
HR_HD uint32_t th_sh(uint32_t lay) { return (lay >> 8) & 255u; }
HR_HD uint32_t bl_sh(uint32_t lay) { return (lay >> 16) & 255u; }
HR_HD uint32_t thread_mask(uint32_t lay) { return (1u << (bl_sh(lay) - th_sh(lay))) - 1u; }
// The block field keeps K = 32 - bl_sh >= 3 bits (widths are at most 6, 8 and
// 10), of which at most 22 are used, as in the 64-bit word.
HR_HD uint32_t block_mask(uint32_t lay)
{
    return (0xFFFFFFFFu >> bl_sh(lay)) & (g::BLOCK_LIMIT - 1u);
}

// State code (tag | cW << 3 | cB << 5 | cL << 7, the low 9 bits of the
// 64-bit word) of each state number, seven 9-bit codes per constant:
//   0 INIT, 1 RACE, 2-3 MB(R/A), 4-7 MW(k, cL) for k = R, A and cL = k, X,
//   8-13 MT and 14-19 ST with cW = R, A and (cB, cL) = (cW,cW), (cW,X), (X,X),
//   20 ST(X, X, X).
constexpr uint64_t code7(uint32_t a, uint32_t b, uint32_t c_, uint32_t d, uint32_t e, uint32_t f,
                         uint32_t h)
{
    return (uint64_t)a | ((uint64_t)b << 9) | ((uint64_t)c_ << 18) | ((uint64_t)d << 27) |
           ((uint64_t)e << 36) | ((uint64_t)f << 45) | ((uint64_t)h << 54);
}
constexpr uint32_t sc(uint32_t tag, uint32_t cl, uint32_t cb, uint32_t cw)
{
    return tag | (cw << 3) | (cb << 5) | (cl << 7);
}
constexpr uint64_t CODES0 = code7(0, T_RACE, sc(T_MB, 0, CL_R, 0), sc(T_MB, 0, CL_A, 0),
                                  sc(T_MW, CL_R, CL_R, 0), sc(T_MW, CL_X, CL_R, 0),
                                  sc(T_MW, CL_A, CL_A, 0));
constexpr uint64_t CODES1 = code7(sc(T_MW, CL_X, CL_A, 0), sc(T_MT, CL_R, CL_R, CL_R),
                                  sc(T_MT, CL_X, CL_R, CL_R), sc(T_MT, CL_X, CL_X, CL_R),
                                  sc(T_MT, CL_A, CL_A, CL_A), sc(T_MT, CL_X, CL_A, CL_A),
                                  sc(T_MT, CL_X, CL_X, CL_A));
constexpr uint64_t CODES2 = code7(sc(T_ST, CL_R, CL_R, CL_R), sc(T_ST, CL_X, CL_R, CL_R),
                                  sc(T_ST, CL_X, CL_X, CL_R), sc(T_ST, CL_A, CL_A, CL_A),
                                  sc(T_ST, CL_X, CL_A, CL_A), sc(T_ST, CL_X, CL_X, CL_A),
                                  sc(T_ST, CL_X, CL_X, CL_X));

HR_HD uint32_t code_of(uint32_t idx)
{
    const uint64_t tbl = idx < 7 ? CODES0 : (idx < 14 ? CODES1 : CODES2);
    const uint32_t j = idx < 7 ? idx : (idx < 14 ? idx - 7 : idx - 14);
    return (uint32_t)(tbl >> (9 * j)) & 511u;
}

// State number of a state code (the inverse of code_of on the 21 codes).
HR_HD uint32_t index_of(uint32_t code)
{
    const uint32_t tag = code & 7u, cw = (code >> 3) & 3u, cb = (code >> 5) & 3u,
                   cl = (code >> 7) & 3u;
    const uint32_t nx = (cl == CL_X ? 1u : 0u) + (cb == CL_X ? 1u : 0u);
    if (tag <= T_RACE) return tag;
    if (tag == T_MB) return 1u + cb;
    if (tag == T_MW) return 4u + 2u * (cb - 1u) + (cl == CL_X ? 1u : 0u);
    if (tag == T_MT) return 8u + 3u * (cw - 1u) + nx;
    return cw == CL_X ? 20u : 14u + 3u * (cw - 1u) + nx;
}

// 32-bit word -> 64-bit word of the same summary.
HR_HD uint64_t widen(uint32_t w, uint32_t lay)
{
    const uint32_t bs = bc_sh(lay), ts = th_sh(lay), ls = bl_sh(lay);
    const uint32_t wc = (w >> WC_SH) & ((1u << (bs - WC_SH)) - 1u);
    const uint32_t bc = (w >> bs) & ((1u << (ts - bs)) - 1u);
    const uint32_t th = (w >> ts) & ((1u << (ls - ts)) - 1u);
    const uint32_t bl = w >> ls;
    return (uint64_t)code_of(w & 31u) | ((uint64_t)wc << g::WC_SH) | ((uint64_t)bc << g::BC_SH) |
           ((uint64_t)th << g::TH_SH) | ((uint64_t)bl << g::BL_SH);
}

// 64-bit word (launch 0, fields within the layout's widths) -> 32-bit word.
HR_HD uint32_t narrow(uint64_t x, uint32_t lay)
{
    const uint32_t wc = (uint32_t)(x >> g::WC_SH) & 63u;
    const uint32_t bc = (uint32_t)(x >> g::BC_SH) & 255u;
    const uint32_t th = (uint32_t)(x >> g::TH_SH) & 1023u;
    const uint32_t bl = (uint32_t)(x >> g::BL_SH) & (g::BLOCK_LIMIT - 1u);
    return index_of((uint32_t)x & 511u) | (wc << WC_SH) | (bc << bc_sh(lay)) |
           (th << th_sh(lay)) | (bl << bl_sh(lay));
}

// Identity fields of an access in the 64-bit layout, block and thread folded
// to the 32-bit word's widths and launch 0.
HR_HD uint64_t pack_id(uint32_t block, uint32_t thread, uint32_t bc, uint32_t wc, uint32_t lay)
{
    return g::pack_id(0, block & block_mask(lay), thread & thread_mask(lay), bc, wc);
}

// The same identity in the 32-bit layout (clocks within their fields).
HR_HD uint32_t pack_id32(uint32_t block, uint32_t thread, uint32_t bc, uint32_t wc, uint32_t lay)
{
    return ((block & block_mask(lay)) << bl_sh(lay)) | ((thread & thread_mask(lay)) << th_sh(lay)) |
           (bc << bc_sh(lay)) | (wc << WC_SH);
}

// Mask of the group (wave or tile) bits of the 32-bit thread field.
HR_HD uint32_t group_mask(uint32_t s, uint32_t lay)
{
    return ((thread_mask(lay) >> s) << s) << th_sh(lay);
}

// State numbers of the multi-accessor and single-thread states (the classes
// form a chain, as every reachable state's do).
HR_HD uint32_t n_of(uint32_t base, uint32_t mul, uint32_t lo, uint32_t nx)
{
    return base + mul * (lo - 1u) + nx;
}
HR_HD uint32_t st_num(uint32_t cl, uint32_t cb, uint32_t cw)
{
    return cw == CL_X ? 20u : n_of(14u, 3u, cw, (cl == CL_X) + (cb == CL_X));
}

// One transition on the 32-bit word: the 64-bit machine's step (g::step)
// written over the 32-bit fields, so that no word is widened on the hook's
// path.  id = pack_id32 of the access; wm = group_mask(s, lay).  It equals
// narrow(g::step(widen(old), pack_id(...), k, g::group_mask(s))).
HR_HD uint32_t step(uint32_t old, uint32_t id, uint32_t k, uint32_t wm, uint32_t lay)
{
    const uint32_t idx = old & 31u;
    if (idx == T_RACE) return old;
    const uint32_t code = code_of(idx);
    const uint32_t tag = code & 7u, cw = (code >> 3) & 3u, cb = (code >> 5) & 3u,
                   cl = (code >> 7) & 3u;
    const uint32_t bs = bc_sh(lay), ts = th_sh(lay), ls = bl_sh(lay);
    const uint32_t wc_m = ((1u << (bs - WC_SH)) - 1u) << WC_SH;
    const uint32_t bc_m = ((1u << (ts - bs)) - 1u) << bs;
    const uint32_t th_m = ((1u << (ls - ts)) - 1u) << ts;
    const uint32_t bl_m = block_mask(lay) << ls;
    const uint32_t d = old ^ id;
    const uint32_t race = T_RACE;
    const uint32_t keep_t = bl_m | bc_m | th_m | wc_m;   // ST
    const uint32_t keep_w = bl_m | bc_m | wm | wc_m;     // MT
    const uint32_t keep_b = bl_m | bc_m;                 // MW
    if (idx == 0) return st_num(k, k, k) | (id & keep_t);
    if (tag == T_MB) return conflicts(cb, k) ? race : old;
    if (d & bl_m) return conflicts(cl, k) ? race : 1u + k;                  // MB(k)
    if (d & bc_m) return st_num(cl | k, k, k) | (id & keep_t);
    if (tag == T_MW) return conflicts(cb, k) ? race : old;
    if (d & wm) return conflicts(cb, k) ? race : (n_of(4u, 2u, k, cl == CL_X) | (id & keep_b));
    if (d & wc_m) return st_num(cl | k, cb | k, k) | (id & keep_t);
    if (tag == T_MT) return conflicts(cw, k) ? race : old;
    if (d & (th_m & ~wm))
        return conflicts(cw, k) ? race
                                : (n_of(8u, 3u, k, (cl == CL_X) + (cb == CL_X)) | (id & keep_w));
    return st_num(cl | k, cb | k, cw | k) | (id & keep_t);
}

HR_HD uint32_t merge(uint32_t x, uint32_t y, uint64_t wm, uint32_t lay)
{
    return narrow(g::merge(widen(x, lay), widen(y, lay), wm), lay);
}
}  // namespace c

// ---------------------------------------------------------------------------
// LDS shadow word, 32 bits: tag 3 | cW 2 | cB 2 | wc 6 | bc 8 | thread 10.
// LDS is private to one block and one launch, so there is no launch, block,
// multi-block state or launch-wide class.
// ---------------------------------------------------------------------------
namespace l {
constexpr uint32_t TAG_SH = 0, CW_SH = 3, CB_SH = 5, WC_SH = 7, BC_SH = 13, TH_SH = 21;
constexpr uint32_t TAG_M = 7u << TAG_SH;
constexpr uint32_t WC_M = 63u << WC_SH;
constexpr uint32_t BC_M = 255u << BC_SH;
constexpr uint32_t TH_M = 1023u << TH_SH;
constexpr uint32_t LANE_M = 63u << TH_SH;
constexpr uint32_t WAVE_M = 15u << (TH_SH + 6);

HR_HD uint32_t group_mask(uint32_t s) { return ((1023u >> s) << s) << TH_SH; }

HR_HD uint32_t pack_id(uint32_t thread, uint32_t bc, uint32_t wc)
{
    return ((thread & 1023u) << TH_SH) | ((bc & 255u) << BC_SH) | ((wc & 63u) << WC_SH);
}

HR_HD uint32_t mk(uint32_t tag, uint32_t cb, uint32_t cw)
{
    return (tag << TAG_SH) | (cb << CB_SH) | (cw << CW_SH);
}

HR_HD uint32_t step(uint32_t old, uint32_t id, uint32_t k, uint32_t wm = WAVE_M)
{
    const uint32_t tag = old & TAG_M;
    if (tag == T_RACE) return old;
    const uint32_t d = old ^ id;
    const uint32_t cb = (old >> CB_SH) & 3u;
    const uint32_t cw = (old >> CW_SH) & 3u;
    const uint32_t race = T_RACE;
    const uint32_t lm = TH_M & ~wm;
    const uint32_t keep_t = BC_M | TH_M | WC_M;
    const uint32_t keep_w = BC_M | wm | WC_M;
    const uint32_t keep_b = BC_M;
    if (tag == T_INIT || (d & BC_M)) return mk(T_ST, k, k) | (id & keep_t);
    if (tag == T_MW) return conflicts(cb, k) ? race : old;
    if (d & wm) return conflicts(cb, k) ? race : (mk(T_MW, k, 0) | (id & keep_b));
    if (d & WC_M) return mk(T_ST, cb | k, k) | (id & keep_t);
    if (tag == T_MT) return conflicts(cw, k) ? race : old;
    if (d & lm) return conflicts(cw, k) ? race : (mk(T_MT, cb, k) | (id & keep_w));
    return mk(T_ST, cb | k, cw | k) | (id & keep_t);
}
}  // namespace l

// ---------------------------------------------------------------------------
// Tiles nested in waves.  The paper leaves synchronization below the warp to
// future work (Sec. VI); cooperative-groups tiles give every aligned group of
// 2^s lanes (s < 6) its own barrier, used beside wave barriers.  This machine
// adds the tile level between the wave and the thread: a tile barrier
// advances the tile clock tc (restarted by wave and block barriers), and two
// accesses of one tile in one wave epoch are ordered exactly when their tile
// epochs differ.  Summaries gain one scope level:
//   MTI(cL, cB, k)       one wave in the latest block epoch; >= 2 tiles in
//                        its latest wave epoch, all of class k
//   MT(cL, cB, cW, k)    one tile in the latest wave epoch; >= 2 threads in
//                        its latest tile epoch, all of class k
//   ST(cL, cB, cW, cT)   one thread in the latest tile epoch
// besides INIT, RACE, MB(k) and MW(cL, k), with cT <= cW <= cB <= cL.  The
// relation goes one step further: ... other wave, later wave epoch, other
// tile, later tile epoch, other thread, same thread.  The tile of a thread is
// the top 10 - s bits of its index (tile_mask(s)).
//
// Global word, 64 bits, least significant first:
//   tag 3 | cT 2 | cW 2 | cB 2 | cL 2 | tc 4 | wc 4 | bc 6 | thread 10 |
//   block 20 | launch 9
// LDS word, 32 bits: tag 3 | cT 2 | cW 2 | cB 2 | tc 4 | wc 4 | bc 5 | thread 10
// (the nested mode bounds the block clock at 5 bits, the wave and tile
// clocks at 4, and launches at 2^20 blocks).
// ---------------------------------------------------------------------------
enum : uint32_t { T_MTI = 6u };

namespace n {
constexpr uint32_t TAG_SH = 0, CT_SH = 3, CW_SH = 5, CB_SH = 7, CL_SH = 9, TC_SH = 11, WC_SH = 15,
                   BC_SH = 19, TH_SH = 25, BL_SH = 35, LA_SH = 55;
constexpr uint64_t TAG_M = 7ull;
constexpr uint64_t CT_M = 3ull << CT_SH, CW_M = 3ull << CW_SH, CB_M = 3ull << CB_SH,
                   CL_M = 3ull << CL_SH;
constexpr uint64_t TC_M = 15ull << TC_SH, WC_M = 15ull << WC_SH, BC_M = 63ull << BC_SH;
constexpr uint64_t TH_M = 1023ull << TH_SH;
constexpr uint64_t WAVE_M = 15ull << (TH_SH + 6);
constexpr uint64_t BL_M = ((1ull << 20) - 1) << BL_SH;
constexpr uint64_t LA_M = 511ull << LA_SH;
constexpr uint32_t BLOCK_LIMIT = 1u << 20;
constexpr uint32_t BC_LIMIT = 32, WC_LIMIT = 16, TC_LIMIT = 16;   // clock values that fit

// Mask of the thread bits naming the tile (tiles of 2^s lanes, s < 6).
HR_HD uint64_t tile_mask(uint32_t s) { return (uint64_t)((1023u >> s) << s) << TH_SH; }

HR_HD uint64_t pack_id(uint32_t launch, uint32_t block, uint32_t thread, uint32_t bc, uint32_t wc,
                       uint32_t tc)
{
    return ((uint64_t)(launch & 511u) << LA_SH) | ((uint64_t)(block & (BLOCK_LIMIT - 1)) << BL_SH) |
           ((uint64_t)(thread & 1023u) << TH_SH) | ((uint64_t)(bc & 63u) << BC_SH) |
           ((uint64_t)(wc & 15u) << WC_SH) | ((uint64_t)(tc & 15u) << TC_SH);
}

HR_HD uint64_t mk(uint32_t tag, uint32_t cl, uint32_t cb, uint32_t cw, uint32_t ct)
{
    return (uint64_t)tag | ((uint64_t)cl << CL_SH) | ((uint64_t)cb << CB_SH) |
           ((uint64_t)cw << CW_SH) | ((uint64_t)ct << CT_SH);
}

// One transition: old word, identity of the access, its class k, and the
// tile mask tm = tile_mask(s).
HR_HD uint64_t step(uint64_t old, uint64_t id, uint32_t k, uint64_t tm)
{
    const uint32_t tag = (uint32_t)(old & TAG_M);
    if (tag == T_RACE) return old;
    const uint64_t d = old ^ id;
    const uint32_t cl = (uint32_t)(old >> CL_SH) & 3u, cb = (uint32_t)(old >> CB_SH) & 3u;
    const uint32_t cw = (uint32_t)(old >> CW_SH) & 3u, ct = (uint32_t)(old >> CT_SH) & 3u;
    const uint64_t race = T_RACE;
    const uint64_t keep_b = LA_M | BL_M | BC_M;            // MW
    const uint64_t keep_i = keep_b | WAVE_M | WC_M;        // MTI
    const uint64_t keep_m = keep_b | tm | WC_M | TC_M;     // MT
    const uint64_t keep_t = keep_b | TH_M | WC_M | TC_M;   // ST
    if (tag == T_INIT || (d & LA_M)) return mk(T_ST, k, k, k, k) | (id & keep_t);
    if (tag == T_MB) return conflicts(cb, k) ? race : old;
    if (d & BL_M) return conflicts(cl, k) ? race : (mk(T_MB, 0, cl | k, 0, 0) | (id & LA_M));
    if (d & BC_M) return mk(T_ST, cl | k, k, k, k) | (id & keep_t);
    if (tag == T_MW) return conflicts(cb, k) ? race : old;
    if (d & WAVE_M) return conflicts(cb, k) ? race : (mk(T_MW, cl, k, 0, 0) | (id & keep_b));
    if (d & WC_M) return mk(T_ST, cl | k, cb | k, k, k) | (id & keep_t);
    if (tag == T_MTI) return conflicts(cw, k) ? race : old;
    if (d & tm) return conflicts(cw, k) ? race : (mk(T_MTI, cl, cb, k, 0) | (id & keep_i));
    if (d & TC_M) return mk(T_ST, cl | k, cb | k, cw | k, k) | (id & keep_t);
    if (tag == T_MT) return conflicts(ct, k) ? race : old;
    if (d & TH_M) return conflicts(ct, k) ? race : (mk(T_MT, cl, cb, cw, k) | (id & keep_m));
    return mk(T_ST, cl | k, cb | k, cw | k, ct | k) | (id & keep_t);
}

// The summary of the union of the access sets of x and y (x of the current
// launch), under the same condition as g::merge, one scope level deeper.
HR_HD uint64_t merge(uint64_t x, uint64_t y, uint64_t tm)
{
    const uint32_t tx = (uint32_t)(x & TAG_M), ty = (uint32_t)(y & TAG_M);
    const uint64_t race = T_RACE;
    if (tx == T_RACE || ty == T_RACE) return race;
    if (ty == T_INIT || ((x ^ y) & LA_M)) return x;
    if (tx == T_INIT) return y;
    const auto cls = [](uint64_t w, uint32_t sh) { return (uint32_t)(w >> sh) & 3u; };
    const uint64_t d = x ^ y;
    if (tx == T_MB || ty == T_MB || (d & BL_M)) {
        const uint32_t c = (tx == T_MB ? cls(x, CB_SH) : cls(x, CL_SH)) |
                           (ty == T_MB ? cls(y, CB_SH) : cls(y, CL_SH));
        return c == CL_X ? race : (mk(T_MB, 0, c, 0, 0) | (x & LA_M));
    }
    const uint32_t cl = cls(x, CL_SH) | cls(y, CL_SH);
    // an earlier epoch at any level is ordered before the newer one, which
    // keeps its detail (clocks never wrap: an overflow stops checking)
    if (d & BC_M) {
        const uint64_t nw = (x & BC_M) > (y & BC_M) ? x : y;
        return (nw & ~CL_M) | ((uint64_t)cl << CL_SH);
    }
    const uint64_t keep_b = LA_M | BL_M | BC_M;
    if (tx == T_MW || ty == T_MW || (d & WAVE_M)) {
        const uint32_t c = cls(x, CB_SH) | cls(y, CB_SH);
        return c == CL_X ? race : (mk(T_MW, cl, c, 0, 0) | (x & keep_b));
    }
    const uint32_t cb = cls(x, CB_SH) | cls(y, CB_SH);
    if (d & WC_M) {
        const uint64_t nw = (x & WC_M) > (y & WC_M) ? x : y;
        return (nw & ~(CL_M | CB_M)) | ((uint64_t)cl << CL_SH) | ((uint64_t)cb << CB_SH);
    }
    if (tx == T_MTI || ty == T_MTI || (d & tm)) {
        const uint32_t c = cls(x, CW_SH) | cls(y, CW_SH);
        return c == CL_X ? race : (mk(T_MTI, cl, cb, c, 0) | (x & (keep_b | WAVE_M | WC_M)));
    }
    const uint32_t cw = cls(x, CW_SH) | cls(y, CW_SH);
    if (d & TC_M) {
        const uint64_t nw = (x & TC_M) > (y & TC_M) ? x : y;
        return (nw & ~(CL_M | CB_M | CW_M)) | ((uint64_t)cl << CL_SH) | ((uint64_t)cb << CB_SH) |
               ((uint64_t)cw << CW_SH);
    }
    if (tx == T_MT || ty == T_MT || (d & TH_M)) {
        const uint32_t c = cls(x, CT_SH) | cls(y, CT_SH);
        return c == CL_X ? race : (mk(T_MT, cl, cb, cw, c) | (x & (keep_b | tm | WC_M | TC_M)));
    }
    return mk(T_ST, cl, cb, cw, cls(x, CT_SH) | cls(y, CT_SH)) |
           (x & (keep_b | TH_M | WC_M | TC_M));
}
}  // namespace n

namespace nl {
constexpr uint32_t TAG_SH = 0, CT_SH = 3, CW_SH = 5, CB_SH = 7, TC_SH = 9, WC_SH = 13, BC_SH = 17,
                   TH_SH = 22;
constexpr uint32_t TAG_M = 7u;
constexpr uint32_t TC_M = 15u << TC_SH, WC_M = 15u << WC_SH, BC_M = 31u << BC_SH;
constexpr uint32_t TH_M = 1023u << TH_SH;
constexpr uint32_t WAVE_M = 15u << (TH_SH + 6);

HR_HD uint32_t tile_mask(uint32_t s) { return ((1023u >> s) << s) << TH_SH; }

HR_HD uint32_t pack_id(uint32_t thread, uint32_t bc, uint32_t wc, uint32_t tc)
{
    return ((thread & 1023u) << TH_SH) | ((bc & 31u) << BC_SH) | ((wc & 15u) << WC_SH) |
           ((tc & 15u) << TC_SH);
}

HR_HD uint32_t mk(uint32_t tag, uint32_t cb, uint32_t cw, uint32_t ct)
{
    return tag | (cb << CB_SH) | (cw << CW_SH) | (ct << CT_SH);
}

// One transition on an LDS word (one block, one launch: no launch, block or
// launch-wide class).
HR_HD uint32_t step(uint32_t old, uint32_t id, uint32_t k, uint32_t tm)
{
    const uint32_t tag = old & TAG_M;
    if (tag == T_RACE) return old;
    const uint32_t d = old ^ id;
    const uint32_t cb = (old >> CB_SH) & 3u, cw = (old >> CW_SH) & 3u, ct = (old >> CT_SH) & 3u;
    const uint32_t race = T_RACE;
    const uint32_t keep_t = BC_M | TH_M | WC_M | TC_M;
    if (tag == T_INIT || (d & BC_M)) return mk(T_ST, k, k, k) | (id & keep_t);
    if (tag == T_MW) return conflicts(cb, k) ? race : old;
    if (d & WAVE_M) return conflicts(cb, k) ? race : (mk(T_MW, k, 0, 0) | (id & BC_M));
    if (d & WC_M) return mk(T_ST, cb | k, k, k) | (id & keep_t);
    if (tag == T_MTI) return conflicts(cw, k) ? race : old;
    if (d & tm)
        return conflicts(cw, k) ? race : (mk(T_MTI, cb, k, 0) | (id & (BC_M | WAVE_M | WC_M)));
    if (d & TC_M) return mk(T_ST, cb | k, cw | k, k) | (id & keep_t);
    if (tag == T_MT) return conflicts(ct, k) ? race : old;
    if (d & TH_M)
        return conflicts(ct, k) ? race : (mk(T_MT, cb, cw, k) | (id & (BC_M | tm | WC_M | TC_M)));
    return mk(T_ST, cb | k, cw | k, ct | k) | (id & keep_t);
}
}  // namespace nl

}  // namespace hr
