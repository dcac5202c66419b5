// Bodies of the instrumented workloads, as device functions of one logical
// block.  The standalone kernels run one logical block per hardware block;
// the job executors run several logical blocks of one job side by side in a
// larger hardware block (each a group of `T` consecutive threads, a multiple
// of the wave size).  `t` is the thread's index in its logical block; a
// thread with t >= T has no logical block and only takes part in the block
// barriers, which every logical block of a hardware block reaches in the
// same order.  CHECK=false compiles the hooks out (plain kernels).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hr_device.h"

#include "hr_hooks.h"
#include "hr_jacobi.h"

// Tree reduction of in[lb*n .. lb*n+n) (n a power of two, n <= 2T) by T
// threads in LDS: load, then log2(n) halving steps, step s adding
// a[t + (n >> (s+1))] into a[t] for t < n >> (s+1), with a block barrier
// after each step unless s == drop; every thread then writes a[0] to
// out[lb*T + t].  When n < 2T a thread's step-0 operand was loaded by
// another thread, so a barrier also follows the loads.
template <int CHECK, class G = hr_gref>
__device__ void reduce_body(const hr_env& e, const G& gin, const G& gout,
                            const int32_t* __restrict__ in, int32_t* __restrict__ out, uint32_t n,
                            uint32_t T, uint32_t lb, uint32_t t, int32_t drop, int32_t* s,
                            uint32_t* sh, uint32_t lds_id)
{
    const bool act = t < T;
    hr_thread th{};
    if constexpr (CHECK) {
        th = hr_thread_make(e, lb, t);
        if (act)
            for (uint32_t i = t; i < n; i += T) sh[i] = 0;
        __syncthreads();
    }
    const size_t base = (size_t)lb * n;
    const size_t o = (size_t)lb * T + t;
    if (act) {
        // A thread loads at most two input words (n <= 2T), t and t + T.
        // The shadow words of both are loaded together and both exchanges
        // are in flight together: a one-block launch is a chain of round
        // trips, and only this thread touches these words.
        const bool one = t < n, two = t + T < n;
        const typename G::word q0 = one ? hr_gload<CHECK>(th, gin, base + t) : 0;
        const typename G::word q1 = two ? hr_gload<CHECK>(th, gin, base + t + T) : 0;
        const int32_t v0 = one ? in[base + t] : 0;
        const int32_t v1 = two ? in[base + t + T] : 0;
        typename G::pend p0{}, p1{};
        if (one) p0 = hr_gi<0, CHECK, true>(e, th, gin, base + t, HR_SITE_REDUCE_LOAD, q0);
        if (two) p1 = hr_gi<0, CHECK, true>(e, th, gin, base + t + T, HR_SITE_REDUCE_LOAD, q1);
        if (one) {
            hr_l<1, CHECK>(e, th, sh, n, lds_id, t, HR_SITE_REDUCE_STAGE);
            s[t] = v0;
        }
        if (two) {
            hr_l<1, CHECK>(e, th, sh, n, lds_id, t + T, HR_SITE_REDUCE_STAGE);
            s[t + T] = v1;
        }
        hr_gs<0, CHECK>(e, th, gin, p0, base + t, HR_SITE_REDUCE_LOAD);
        hr_gs<0, CHECK>(e, th, gin, p1, base + t + T, HR_SITE_REDUCE_LOAD);
    }
    if (n != 2 * T) hr_bar<CHECK>(e, th);
    const int32_t steps = 31 - __builtin_clz(n);
    for (int32_t step = 0; step < steps; ++step) {
        const uint32_t h = n >> (step + 1);
        if (act && t < h) {
            const int32_t x = s[t];
            const int32_t y = s[t + h];
            s[t] = x + y;
            if constexpr (CHECK)
                hr_lds_rrw<CHECK == 2>(e, th, sh, n, lds_id, t, t + h, HR_SITE_REDUCE_LEFT,
                           HR_SITE_REDUCE_RIGHT, HR_SITE_REDUCE_SUM);
        }
        if (step != drop) hr_bar<CHECK>(e, th);
    }
    if (act) {
        // the output word's shadow load is in flight during the LDS read
        const typename G::word pre_out = hr_gload<CHECK>(th, gout, o);
        const int32_t r = s[0];
        hr_l<0, CHECK>(e, th, sh, n, lds_id, 0, HR_SITE_REDUCE_TOTAL);
        out[o] = r;
        hr_gpre<1, CHECK, false>(e, th, gout, o, HR_SITE_REDUCE_OUT, pre_out);
    }
}

// One logical block (T threads, vertices lb*T .. lb*T+T) of label
// propagation: l = atomic load of label[v]; for every edge (v, u) an atomic
// min of l into label[u], or for a seeded edge a plain read and plain write
// of label[u].  grp / gcol: optional monitoring of the CSR reads (shadow
// null when off).
template <int CHECK, bool PAIRS = false, class G = hr_gref>
__device__ void labelprop_body(const hr_env& e, const G& glab, const G& grp, const G& gcol,
                               int32_t* __restrict__ label, const int32_t* __restrict__ rp,
                               const int32_t* __restrict__ col, const uint8_t* __restrict__ mask,
                               uint32_t n, uint32_t T, uint32_t lb, uint32_t t)
{
    const uint32_t v = lb * T + t;
    if (t >= T || v >= n) return;
    hr_thread th{};
    if constexpr (CHECK) th = hr_thread_make(e, lb, t);
    const int32_t l = __hip_atomic_load(label + v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    hr_g<2, CHECK>(e, th, glab, v, HR_SITE_LP_OWN);
    const int32_t e0 = rp[v], e1 = rp[v + 1];
    if (CHECK && grp.shadow) {
        hr_g<0, CHECK>(e, th, grp, v, HR_SITE_LP_CSR);
        hr_g<0, CHECK>(e, th, grp, v + 1, HR_SITE_LP_CSR);
    }
    if constexpr (!CHECK) {
        // the plain kernel: nothing to hide, the simple loop is its fastest form
        for (int32_t k = e0; k < e1; ++k) {
            const uint32_t u = (uint32_t)col[k];
            if (u >= n) continue;
            if (mask[k]) {
                const int32_t r = label[u];
                label[u] = r < l ? r : l;
            } else {
                atomicMin(label + u, l);
            }
        }
        return;
    }
    if (PAIRS && !e.group) {
        // Edges in pairs, for the long lists of hub vertices whose threads
        // bound the launch: the exchanges of both edges of a pair are in
        // flight together and settled after both are issued, while the
        // column indices of the pair after next and the seeded flags and
        // shadow words of the next pair are loaded.  (It takes more
        // registers than the batch and serving workers, which inline every
        // workload body, can give; they run the one-edge loop below.)
        const auto col_at = [&](int32_t q) { return q < e1 ? (uint32_t)col[q] : 0u; };
        uint32_t a0 = col_at(e0), b0 = col_at(e0 + 1), a1 = col_at(e0 + 2), b1 = col_at(e0 + 3);
        typename G::word sa = e0 < e1 ? hr_gload<CHECK>(th, glab, a0) : 0;
        typename G::word sb = e0 + 1 < e1 ? hr_gload<CHECK>(th, glab, b0) : 0;
        uint8_t ma = e0 < e1 ? mask[e0] : 0, mb = e0 + 1 < e1 ? mask[e0 + 1] : 0;
        for (int32_t k = e0; k < e1; k += 2) {
            const uint32_t a2 = col_at(k + 4), b2 = col_at(k + 5);
            const typename G::word na = k + 2 < e1 ? hr_gload<CHECK>(th, glab, a1) : 0;
            const typename G::word nb = k + 3 < e1 ? hr_gload<CHECK>(th, glab, b1) : 0;
            const uint8_t nma = k + 2 < e1 ? mask[k + 2] : 0, nmb = k + 3 < e1 ? mask[k + 3] : 0;
            const uint32_t ua = a0, ub = b0;
            const typename G::word qa = sa, qb = sb;
            const uint8_t fa = ma, fb = mb;
            const bool two = k + 1 < e1;
            a0 = a1;
            b0 = b1;
            a1 = a2;
            b1 = b2;
            sa = na;
            sb = nb;
            ma = nma;
            mb = nmb;
            if (gcol.shadow) {
                hr_g<0, CHECK>(e, th, gcol, (uint64_t)k, HR_SITE_LP_CSR);
                if (two) hr_g<0, CHECK>(e, th, gcol, (uint64_t)k + 1, HR_SITE_LP_CSR);
            }
            typename G::pend pa{}, pb{};
            if (ua < n) {
                if (fa) {
                    const int32_t r = label[ua];
                    hr_gpre<0, CHECK>(e, th, glab, ua, HR_SITE_LP_SEED_READ, qa);
                    label[ua] = r < l ? r : l;
                    hr_g<1, CHECK, true>(e, th, glab, ua, HR_SITE_LP_SEED_WRITE);
                } else {
                    atomicMin(label + ua, l);
                    pa = hr_gi<2, CHECK, true>(e, th, glab, ua, HR_SITE_LP_MIN, qa);
                }
            }
            if (two && ub < n) {
                if (fb) {
                    const int32_t r = label[ub];
                    hr_gpre<0, CHECK>(e, th, glab, ub, HR_SITE_LP_SEED_READ, qb);
                    label[ub] = r < l ? r : l;
                    hr_g<1, CHECK, true>(e, th, glab, ub, HR_SITE_LP_SEED_WRITE);
                } else {
                    atomicMin(label + ub, l);
                    pb = hr_gi<2, CHECK, true>(e, th, glab, ub, HR_SITE_LP_MIN, qb);
                }
            }
            hr_gs<2, CHECK>(e, th, glab, pa, ua, HR_SITE_LP_MIN);
            hr_gs<2, CHECK>(e, th, glab, pb, ub, HR_SITE_LP_MIN);
        }
        return;
    }
    // One edge at a time.  While edge k is checked, the
    // column index of edge k+2, and the seeded flag of edge k+1 and the
    // shadow word of its target, are already in flight.
    uint32_t u0 = e0 < e1 ? (uint32_t)col[e0] : 0u;
    uint32_t u1 = e0 + 1 < e1 ? (uint32_t)col[e0 + 1] : 0u;
    typename G::word s0 = e0 < e1 ? hr_gload<CHECK>(th, glab, u0) : 0;
    uint8_t m0 = e0 < e1 ? mask[e0] : 0;
    for (int32_t k = e0; k < e1; ++k) {
        const uint32_t u2 = k + 2 < e1 ? (uint32_t)col[k + 2] : 0u;
        const typename G::word s1 = k + 1 < e1 ? hr_gload<CHECK>(th, glab, u1) : 0;
        const uint8_t m1 = k + 1 < e1 ? mask[k + 1] : 0;
        const uint32_t u = u0;
        const typename G::word su = s0;
        const uint8_t seeded = m0;
        u0 = u1;
        u1 = u2;
        s0 = s1;
        m0 = m1;
        if (CHECK && gcol.shadow) hr_g<0, CHECK>(e, th, gcol, (uint64_t)k, HR_SITE_LP_CSR);
        if (u >= n) continue;
        if (seeded) {
            const int32_t r = label[u];
            hr_gpre<0, CHECK>(e, th, glab, u, HR_SITE_LP_SEED_READ, su);
            label[u] = r < l ? r : l;
            hr_g<1, CHECK, true>(e, th, glab, u, HR_SITE_LP_SEED_WRITE);
        } else {
            atomicMin(label + u, l);
            hr_gpre<2, CHECK>(e, th, glab, u, HR_SITE_LP_MIN, su);
        }
    }
}
