// Standalone instrumented workloads (one logical block per hardware block),
// the access-program interpreter, and their launchers.  Each workload kernel
// is a template on CHECK so the plain kernel is the same code with the hooks
// compiled out.
#include <hip/hip_runtime.h>

#include "hr.h"
#include "hr_bodies.h"
#include "hr_device.h"
#include "hr_internal.h"
#include "hr_nested.h"

namespace {

// The hooks' view of kernel-argument region r.  cols: the row width a 2-D
// workload indexes the region with, which is the width of a row-major map
// (a tiled map carries its own and must agree; the launchers check that).
hr_gref gref(const hr_kargs& a, uint32_t r, uint32_t cols = 0)
{
    hr_gref g{nullptr, 0, r, hr_lay_rows(cols)};
    if (r < HR_MAX_REGIONS) {
        g.shadow = a.shadow[r];
        g.n = a.n_elems[r];
        if (a.lay[r].tw | a.lay[r].th) g.lay = a.lay[r];
    }
    return g;
}

template <uint32_t LAY = 0>
hr_gref4t<LAY> gref4(const hr_kargs& a, uint32_t r, uint32_t cols = 0)
{
    hr_gref4t<LAY> g{nullptr, 0, r, hr_lay_rows(cols)};
    if (r < HR_MAX_REGIONS) {
        g.shadow = (uint32_t*)a.shadow[r];
        g.n = a.n_elems[r];
        if (a.lay[r].tw | a.lay[r].th) g.lay = a.lay[r];
    }
    return g;
}

// A region's map is the row-major identity (what the 1-D workloads assume).
bool lay_flat(const hr_kargs& a, uint32_t r)
{
    return r >= HR_MAX_REGIONS || (a.lay[r].tw | a.lay[r].th) == 0;
}

// A region's map fits a 2-D workload nx elements wide: row-major, or tiled
// over rows of exactly nx elements.
bool lay_fits(const hr_kargs& a, uint32_t r, uint32_t nx)
{
    if (r >= HR_MAX_REGIONS) return false;
    const hr_lay& L = a.lay[r];
    return (L.tw | L.th) == 0 || L.cols == nx;
}

// CHECK 0: plain, 1: checked, 2: checked with the debug access log.
template <int CHECK>
__global__ __launch_bounds__(1024) void k_reduce(hr_kargs a, hr_gref gin, hr_gref gout,
                                                 const int32_t* __restrict__ in,
                                                 int32_t* __restrict__ out, uint32_t n,
                                                 int32_t drop)
{
    extern __shared__ uint32_t smem[];
    using G = hr_gref_1d;
    reduce_body<CHECK>(a.env, G{gin}, G{gout}, in, out, n, blockDim.x, blockIdx.x, threadIdx.x,
                       drop, (int32_t*)smem, smem + n, 0);
}

template <int CHECK>
__global__ __launch_bounds__(1024) void k_labelprop(hr_kargs a, hr_gref glab, hr_gref grp,
                                                    hr_gref gcol, int32_t* __restrict__ label,
                                                    const int32_t* __restrict__ rp,
                                                    const int32_t* __restrict__ col,
                                                    const uint8_t* __restrict__ mask, uint32_t n)
{
    using G = hr_gref_1d;
    labelprop_body<CHECK, true, G>(a.env, G{glab}, G{grp}, G{gcol}, label, rp, col, mask, n,
                                   blockDim.x, blockIdx.x, threadIdx.x);
}

// The checked kernels on 4-byte shadow words.
template <int CHECK = 1>
__global__ __launch_bounds__(1024) void k_reduce4(hr_kargs a, hr_gref4 gin, hr_gref4 gout,
                                                  const int32_t* __restrict__ in,
                                                  int32_t* __restrict__ out, uint32_t n,
                                                  int32_t drop)
{
    extern __shared__ uint32_t smem[];
    using G = hr_gref4_1d<0>;
    reduce_body<CHECK>(a.env, G{gin}, G{gout}, in, out, n, blockDim.x, blockIdx.x, threadIdx.x,
                       drop, (int32_t*)smem, smem + n, 0);
}

template <int CHECK = 1>
__global__ __launch_bounds__(1024) void k_labelprop4(hr_kargs a, hr_gref4 glab, hr_gref4 grp,
                                                     hr_gref4 gcol, int32_t* __restrict__ label,
                                                     const int32_t* __restrict__ rp,
                                                     const int32_t* __restrict__ col,
                                                     const uint8_t* __restrict__ mask, uint32_t n)
{
    using G = hr_gref4_1d<0>;
    labelprop_body<CHECK, true, G>(a.env, G{glab}, G{grp}, G{gcol}, label, rp, col, mask, n,
                                   blockDim.x, blockIdx.x, threadIdx.x);
}

// ----------------------------------------------------------- interpreter
struct prog_map {
    uint32_t r[8];
};

// TABLE: global transitions from the flat table at tab (HR_CFG_FSM_TABLE).
template <bool LOG = false, bool TABLE = false>
__global__ __launch_bounds__(1024) void k_program(hr_kargs a, prog_map pm, uint32_t blocks,
                                                  uint32_t threads, uint32_t phases,
                                                  const uint8_t* __restrict__ scope,
                                                  const uint64_t* __restrict__ wmask,
                                                  const int32_t* __restrict__ op_off,
                                                  size_t n_op_off, const uint32_t* __restrict__ ops,
                                                  size_t n_ops, const uint32_t* __restrict__ bmap,
                                                  uint32_t lds_words, const uint16_t* tab)
{
    extern __shared__ uint32_t smem[];
    uint32_t* ldata = smem;
    uint32_t* lsh = smem + lds_words;
    const uint32_t b = bmap ? bmap[blockIdx.x] : blockIdx.x;
    if (b >= blocks) return;                      // uniform over the block
    const uint32_t t = threadIdx.x;
    hr_thread th = hr_thread_make(a.env, b, t);
    for (uint32_t i = t; i < lds_words; i += blockDim.x) {
        ldata[i] = 0;
        lsh[i] = 0;
    }
    __syncthreads();
    const uint32_t w = t >> a.env.wave_bits;     // the thread's wave, or tile
    for (uint32_t p = 0; p < phases; ++p) {
        const size_t i = ((size_t)p * blocks + b) * threads + t;
        int64_t k0 = 0, k1 = 0;
        if (i + 1 < n_op_off) {
            k0 = op_off[i];
            k1 = op_off[i + 1];
        }
        if (k0 < 0) k0 = 0;
        if (k1 > (int64_t)n_ops) k1 = (int64_t)n_ops;
        for (int64_t k = k0; k < k1; ++k) {
            const uint32_t op = ops[k];
            const uint32_t idx = op & 0xFFFFFFu, reg = (op >> 24) & 7u, kind = (op >> 27) & 3u;
            if (kind == 3) {                        // switch this thread's checking
                hr_thread_enable(th, idx & 1u);
                continue;
            }
            if ((op >> 29) & 1u) {
                if (idx >= lds_words) {
                    hr_set_flag(a.env, HR_DEVF_RANGE);
                    continue;
                }
                if (kind == 0) (void)*(volatile uint32_t*)(ldata + idx);
                else if (kind == 1) ldata[idx] = t + 1;
                else atomicAdd(ldata + idx, 1u);
                hr_access_lds_k<LOG>(a.env, th, kind, lsh, lds_words, 0, idx, p + 1);
            } else {
                const uint32_t r = pm.r[reg];
                if (r >= HR_MAX_REGIONS || idx >= a.n_elems[r]) {
                    hr_set_flag(a.env, HR_DEVF_RANGE);
                    continue;
                }
                uint32_t* d = (uint32_t*)a.data[r];
                if (kind == 0) (void)*(volatile uint32_t*)(d + idx);
                else if (kind == 1) d[idx] = t + 1;
                else atomicAdd(d + idx, 1u);
                hr_check_k<LOG, TABLE>(a.env, th, kind, a.shadow[r], a.n_elems[r], r, idx,
                                       hr_lay_off(a.lay[r], idx), p + 1, tab);
            }
        }
        const uint8_t sc = scope[p];
        if (sc == 2) hr_barrier_block(a.env, th);
        else if (sc == 1 && w < 64 && ((wmask[p] >> w) & 1ull)) hr_barrier_wave(a.env, th);
    }
}

// The interpreter on the nested machine: tiles of 2^wave_bits lanes inside
// 64-lane waves.  A phase ends with nothing (scope 0), a wave barrier in the
// waves whose bit is set in wmask[p] (scope 1), a block barrier (scope 2) or
// a tile barrier in the tiles whose bit is set in wmask[p] (scope 3; tiles
// past the 64th never synchronize).
template <bool LOG = false>
__global__ __launch_bounds__(1024) void k_program_nested(
    hr_kargs a, prog_map pm, uint32_t blocks, uint32_t threads, uint32_t phases,
    const uint8_t* __restrict__ scope, const uint64_t* __restrict__ wmask,
    const int32_t* __restrict__ op_off, size_t n_op_off, const uint32_t* __restrict__ ops,
    size_t n_ops, const uint32_t* __restrict__ bmap, uint32_t lds_words)
{
    extern __shared__ uint32_t smem[];
    uint32_t* ldata = smem;
    uint32_t* lsh = smem + lds_words;
    const uint32_t b = bmap ? bmap[blockIdx.x] : blockIdx.x;
    if (b >= blocks) return;                      // uniform over the block
    const uint32_t t = threadIdx.x;
    hr_tn th = hr_tn_make(a.env, b, t);
    for (uint32_t i = t; i < lds_words; i += blockDim.x) {
        ldata[i] = 0;
        lsh[i] = 0;
    }
    __syncthreads();
    const uint32_t w = t >> 6, g = t >> a.env.wave_bits;   // the thread's wave and tile
    for (uint32_t p = 0; p < phases; ++p) {
        const size_t i = ((size_t)p * blocks + b) * threads + t;
        int64_t k0 = 0, k1 = 0;
        if (i + 1 < n_op_off) {
            k0 = op_off[i];
            k1 = op_off[i + 1];
        }
        if (k0 < 0) k0 = 0;
        if (k1 > (int64_t)n_ops) k1 = (int64_t)n_ops;
        for (int64_t k = k0; k < k1; ++k) {
            const uint32_t op = ops[k];
            const uint32_t idx = op & 0xFFFFFFu, reg = (op >> 24) & 7u, kind = (op >> 27) & 3u;
            if (kind == 3) {
                hr_tn_enable(th, idx & 1u);
                continue;
            }
            if ((op >> 29) & 1u) {
                if (idx >= lds_words) {
                    hr_set_flag(a.env, HR_DEVF_RANGE);
                    continue;
                }
                if (kind == 0) (void)*(volatile uint32_t*)(ldata + idx);
                else if (kind == 1) ldata[idx] = t + 1;
                else atomicAdd(ldata + idx, 1u);
                hr_naccess_lds_k<LOG>(a.env, th, kind, lsh, lds_words, 0, idx, p + 1);
            } else {
                const uint32_t r = pm.r[reg];
                if (r >= HR_MAX_REGIONS || idx >= a.n_elems[r]) {
                    hr_set_flag(a.env, HR_DEVF_RANGE);
                    continue;
                }
                uint32_t* d = (uint32_t*)a.data[r];
                if (kind == 0) (void)*(volatile uint32_t*)(d + idx);
                else if (kind == 1) d[idx] = t + 1;
                else atomicAdd(d + idx, 1u);
                hr_ncheck_k<LOG>(a.env, th, kind, a.shadow[r], a.n_elems[r], r, idx,
                                 hr_lay_off(a.lay[r], idx), p + 1);
            }
        }
        const uint8_t sc = scope[p];
        if (sc == 2) hr_nbarrier_block(a.env, th);
        else if (sc == 1 && w < 64 && ((wmask[p] >> w) & 1ull)) hr_nbarrier_wave(a.env, th);
        else if (sc == 3 && g < 64 && ((wmask[p] >> g) & 1ull)) hr_nbarrier_tile(a.env, th);
    }
}

}  // namespace

// ======================================================================
static bool reduce_shape_ok(uint32_t n, uint32_t threads, uint32_t blocks)
{
    if (threads == 0 || threads > 1024 || threads % 64 || blocks == 0) return false;
    if (n < 2 || (n & (n - 1)) || n > 2 * threads || n > 8192) return false;
    return blocks < hr::g::BLOCK_LIMIT;
}

extern "C" hr_status hr_reduce_check(hr_ctx c, uint32_t r_in, uint32_t r_out, const int32_t* in_dev,
                                     int32_t* out_dev, uint32_t n, uint32_t threads,
                                     uint32_t blocks, int32_t drop, void* stream)
{
    if (c && (c->cfg.flags & (HR_CFG_NESTED_TILES | HR_CFG_FSM_TABLE)))
        return HR_E_INVAL;   // no tile level, no table form here
    if (!c || !reduce_shape_ok(n, threads, blocks) ||
        !hr_region_ok(c, r_in, in_dev, (size_t)n * blocks) ||
        !hr_region_ok(c, r_out, out_dev, (size_t)threads * blocks))
        return HR_E_INVAL;
    hr_kargs a;
    hr_fill_args(c, &a);
    return hr_launch_reduce(a, r_in, r_out, in_dev, out_dev, n, threads, blocks, drop,
                            hr_stream(c, stream));
}

hr_status hr_launch_reduce(const hr_kargs& a, uint32_t r_in, uint32_t r_out, const int32_t* in_dev,
                           int32_t* out_dev, uint32_t n, uint32_t threads, uint32_t blocks,
                           int32_t drop, hipStream_t s)
{
    if (!in_dev || !out_dev || !reduce_shape_ok(n, threads, blocks)) return HR_E_INVAL;
    if (!lay_flat(a, r_in) || !lay_flat(a, r_out)) return HR_E_INVAL;
    // a context with an access log runs the kernels that write it
    const bool log = a.env.log != nullptr;
    if (a.env.word4)
        HR_LAUNCH(log ? k_reduce4<2> : k_reduce4<1>, dim3(blocks), dim3(threads), (size_t)n * 8, s,
                  a, gref4(a, r_in), gref4(a, r_out), in_dev, out_dev, n, drop);
    else
        HR_LAUNCH(log ? k_reduce<2> : k_reduce<1>, dim3(blocks), dim3(threads), (size_t)n * 8, s,
                  a, gref(a, r_in), gref(a, r_out), in_dev, out_dev, n, drop);
    return HR_OK;
}

extern "C" hr_status hr_reduce_plain(const int32_t* in_dev, int32_t* out_dev, uint32_t n,
                                     uint32_t threads, uint32_t blocks, int32_t drop, void* stream)
{
    if (!in_dev || !out_dev || !reduce_shape_ok(n, threads, blocks)) return HR_E_INVAL;
    hr_kargs a{};
    HR_LAUNCH(k_reduce<0>, dim3(blocks), dim3(threads), (size_t)n * 4, (hipStream_t)stream, a,
              hr_gref{}, hr_gref{}, in_dev, out_dev, n, drop);
    return HR_OK;
}

static bool jacobi_shape_ok(uint32_t ny, uint32_t nx)
{
    if (ny == 0 || nx == 0) return false;
    const uint64_t nbx = (nx + 15) / 16, nby = (ny + 15) / 16;
    return nby <= 65535 && nbx <= 65535 && nbx * nby < hr::g::BLOCK_LIMIT;
}

extern "C" hr_status hr_jacobi_check(hr_ctx c, uint32_t r_old, uint32_t r_new,
                                     const float* u_old_dev, float* u_new_dev, uint32_t ny,
                                     uint32_t nx, const int32_t* seed_dev, void* stream)
{
    if (c && (c->cfg.flags & HR_CFG_NESTED_TILES)) return HR_E_INVAL;   // no tile level here
    if (!c || !jacobi_shape_ok(ny, nx)) return HR_E_INVAL;
    const size_t cells = (size_t)ny * nx;
    if (!hr_region_ok(c, r_old, u_old_dev, cells) || !hr_region_ok(c, r_new, u_new_dev, cells))
        return HR_E_INVAL;
    hr_kargs a;
    hr_fill_args(c, &a);
    if (c->cfg.flags & HR_CFG_FSM_TABLE) {
        // the transitions from the flat table: the row-major kernel only
        if (!c->fsm_tab || !u_old_dev || !u_new_dev || !lay_flat(a, r_old) ||
            !lay_flat(a, r_new) || !lay_fits(a, r_old, nx) || !lay_fits(a, r_new, nx))
            return HR_E_INVAL;
        auto k = (c->cfg.flags & HR_CFG_FSM_TABLE_LDS) ? k_jacobi_tab<1, true> : k_jacobi_tab<1>;
        HR_LAUNCH(k, dim3((nx + 15) / 16, (ny + 15) / 16), dim3(256), 0, hr_stream(c, stream), a,
                  gref(a, r_old, nx), gref(a, r_new, nx), u_old_dev, u_new_dev, ny, nx, seed_dev,
                  (const uint16_t*)c->fsm_tab);
        return HR_OK;
    }
    return hr_launch_jacobi(a, r_old, r_new, u_old_dev, u_new_dev, ny, nx, seed_dev,
                            hr_stream(c, stream));
}

hr_status hr_launch_jacobi(const hr_kargs& a, uint32_t r_old, uint32_t r_new,
                           const float* u_old_dev, float* u_new_dev, uint32_t ny, uint32_t nx,
                           const int32_t* seed_dev, hipStream_t s)
{
    if (!u_old_dev || !u_new_dev || !jacobi_shape_ok(ny, nx)) return HR_E_INVAL;
    if (!lay_fits(a, r_old, nx) || !lay_fits(a, r_new, nx)) return HR_E_INVAL;
    const dim3 grid((nx + 15) / 16, (ny + 15) / 16);
    constexpr uint32_t DL = hr::c::DEFAULT_LAYOUT;
    if (a.env.log && a.env.word4)   // the kernels with the access log: any map
        HR_LAUNCH((k_jacobi4<0, 2>), grid, dim3(256), 0, s, a, gref4(a, r_old, nx),
                  gref4(a, r_new, nx), u_old_dev, u_new_dev, ny, nx, seed_dev);
    else if (a.env.log)
        HR_LAUNCH((k_jacobi_tiled<-1, -1, 2>), grid, dim3(256), 0, s, a, gref(a, r_old, nx),
                  gref(a, r_new, nx), u_old_dev, u_new_dev, ny, nx, seed_dev);
    else if (a.env.word4 == DL)
        HR_LAUNCH(k_jacobi4<DL>, grid, dim3(256), 0, s, a, gref4<DL>(a, r_old, nx),
                  gref4<DL>(a, r_new, nx), u_old_dev, u_new_dev, ny, nx, seed_dev);
    else if (a.env.word4)
        HR_LAUNCH(k_jacobi4<0>, grid, dim3(256), 0, s, a, gref4(a, r_old, nx),
                  gref4(a, r_new, nx), u_old_dev, u_new_dev, ny, nx, seed_dev);
    else {
        // the kernel with the grids' map as a constant when there is one
        const hr_lay &lo = a.lay[r_old], &ln = a.lay[r_new];
        const uint32_t to = lo.tw | lo.th << 4, tn = ln.tw | ln.th << 4;
        auto k = k_jacobi_tiled<-1, -1>;
        if (to == 0 && tn == 0) k = k_jacobi<1>;
        else if (to == tn && to == (2u | 2u << 4)) k = k_jacobi_tiled<2, 2>;
        else if (to == tn && to == (2u | 1u << 4)) k = k_jacobi_tiled<2, 1>;
        else if (to == tn && to == (3u | 1u << 4)) k = k_jacobi_tiled<3, 1>;
        HR_LAUNCH(k, grid, dim3(256), 0, s, a, gref(a, r_old, nx), gref(a, r_new, nx), u_old_dev,
                  u_new_dev, ny, nx, seed_dev);
    }
    return HR_OK;
}

extern "C" hr_status hr_jacobi_plain(const float* u_old_dev, float* u_new_dev, uint32_t ny,
                                     uint32_t nx, const int32_t* seed_dev, void* stream)
{
    if (!u_old_dev || !u_new_dev || !jacobi_shape_ok(ny, nx)) return HR_E_INVAL;
    hr_kargs a{};
    const dim3 grid((nx + 15) / 16, (ny + 15) / 16);
    HR_LAUNCH(k_jacobi<0>, grid, dim3(256), 0, (hipStream_t)stream, a, hr_gref{}, hr_gref{},
              u_old_dev, u_new_dev, ny, nx, seed_dev);
    return HR_OK;
}

static bool labelprop_shape_ok(uint32_t n, uint32_t tpb)
{
    if (n == 0 || tpb == 0 || tpb > 1024) return false;
    return (uint64_t)(n + tpb - 1) / tpb < hr::g::BLOCK_LIMIT;
}

extern "C" hr_status hr_labelprop_check(hr_ctx c, uint32_t r_label, uint32_t r_row_ptr,
                                        uint32_t r_col, int32_t* label_dev,
                                        const int32_t* row_ptr_dev, const int32_t* col_dev,
                                        const uint8_t* mask_dev, uint32_t n, uint32_t tpb,
                                        void* stream)
{
    if (c && (c->cfg.flags & (HR_CFG_NESTED_TILES | HR_CFG_FSM_TABLE)))
        return HR_E_INVAL;   // no tile level, no table form here
    if (!c || !row_ptr_dev || !col_dev || !mask_dev || !labelprop_shape_ok(n, tpb) ||
        !hr_region_ok(c, r_label, label_dev, n))
        return HR_E_INVAL;
    if (r_row_ptr != UINT32_MAX && !hr_region_ok(c, r_row_ptr, row_ptr_dev, (size_t)n + 1))
        return HR_E_INVAL;
    if (r_col != UINT32_MAX && !hr_region_ok(c, r_col, col_dev, 1)) return HR_E_INVAL;
    hr_kargs a;
    hr_fill_args(c, &a);
    return hr_launch_labelprop(a, r_label, r_row_ptr, r_col, label_dev, row_ptr_dev, col_dev,
                               mask_dev, n, tpb, hr_stream(c, stream));
}

hr_status hr_launch_labelprop(const hr_kargs& a, uint32_t r_label, uint32_t r_row_ptr,
                              uint32_t r_col, int32_t* label_dev, const int32_t* row_ptr_dev,
                              const int32_t* col_dev, const uint8_t* mask_dev, uint32_t n,
                              uint32_t tpb, hipStream_t s)
{
    if (!label_dev || !row_ptr_dev || !col_dev || !mask_dev || !labelprop_shape_ok(n, tpb))
        return HR_E_INVAL;
    if (!lay_flat(a, r_label) || !lay_flat(a, r_row_ptr) || !lay_flat(a, r_col))
        return HR_E_INVAL;
    const bool log = a.env.log != nullptr;
    if (a.env.word4) {
        const hr_gref4 none{nullptr, 0, 0};
        HR_LAUNCH(log ? k_labelprop4<2> : k_labelprop4<1>, dim3((n + tpb - 1) / tpb), dim3(tpb),
                  0, s, a, gref4(a, r_label),
                  r_row_ptr != UINT32_MAX ? gref4(a, r_row_ptr) : none,
                  r_col != UINT32_MAX ? gref4(a, r_col) : none, label_dev, row_ptr_dev, col_dev,
                  mask_dev, n);
        return HR_OK;
    }
    const hr_gref none{nullptr, 0, 0};
    HR_LAUNCH(log ? k_labelprop<2> : k_labelprop<1>, dim3((n + tpb - 1) / tpb), dim3(tpb), 0, s,
              a, gref(a, r_label),
              r_row_ptr != UINT32_MAX ? gref(a, r_row_ptr) : none,
              r_col != UINT32_MAX ? gref(a, r_col) : none, label_dev, row_ptr_dev, col_dev,
              mask_dev, n);
    return HR_OK;
}

extern "C" hr_status hr_labelprop_plain(int32_t* label_dev, const int32_t* row_ptr_dev,
                                        const int32_t* col_dev, const uint8_t* mask_dev, uint32_t n,
                                        uint32_t tpb, void* stream)
{
    if (!label_dev || !row_ptr_dev || !col_dev || !mask_dev || !labelprop_shape_ok(n, tpb))
        return HR_E_INVAL;
    hr_kargs a{};
    HR_LAUNCH(k_labelprop<0>, dim3((n + tpb - 1) / tpb), dim3(tpb), 0, (hipStream_t)stream, a,
              hr_gref{}, hr_gref{}, hr_gref{}, label_dev, row_ptr_dev, col_dev, mask_dev, n);
    return HR_OK;
}

extern "C" hr_status hr_program_check(hr_ctx c, const uint32_t* regions_host, uint32_t n_regions,
                                      uint32_t blocks, uint32_t threads, uint32_t phases,
                                      const uint8_t* scope_dev, const uint64_t* wave_mask_dev,
                                      const int32_t* op_off_dev, size_t n_op_off,
                                      const uint32_t* ops_dev, size_t n_ops,
                                      const uint32_t* block_map_dev, uint32_t lds_words,
                                      void* stream)
{
    if (!c || blocks == 0 || threads == 0 || threads > 1024 || lds_words > 8192 ||
        n_regions > 8 || (n_regions && !regions_host) || blocks >= hr::g::BLOCK_LIMIT)
        return HR_E_INVAL;
    if (phases && (!scope_dev || !wave_mask_dev || !op_off_dev)) return HR_E_INVAL;
    if (phases && n_op_off < (size_t)phases * blocks * threads + 1) return HR_E_INVAL;
    if (n_ops && !ops_dev) return HR_E_INVAL;
    prog_map pm;
    for (uint32_t i = 0; i < 8; ++i) pm.r[i] = UINT32_MAX;
    for (uint32_t i = 0; i < n_regions; ++i) {
        if (regions_host[i] >= HR_MAX_REGIONS || regions_host[i] >= c->reg.size() ||
            !c->reg[regions_host[i]].live)
            return HR_E_INVAL;
        pm.r[i] = regions_host[i];
    }
    hr_kargs a;
    hr_fill_args(c, &a);
    const size_t lds_bytes = (size_t)lds_words * 2 * sizeof(uint32_t);
    const bool nested = (c->cfg.flags & HR_CFG_NESTED_TILES) != 0;
    if (nested && blocks > hr::n::BLOCK_LIMIT) return HR_E_INVAL;
    if (nested) {
        auto kern = a.env.log ? k_program_nested<true> : k_program_nested<false>;
        HR_LAUNCH(kern, dim3(blocks), dim3(threads), lds_bytes, hr_stream(c, stream), a, pm,
                  blocks, threads, phases, scope_dev, wave_mask_dev, op_off_dev, n_op_off, ops_dev,
                  n_ops, block_map_dev, lds_words);
        return HR_OK;
    }
    auto kern = a.env.log ? k_program<true> : k_program<false>;
    if (c->fsm_tab) kern = k_program<false, true>;
    HR_LAUNCH(kern, dim3(blocks), dim3(threads), lds_bytes, hr_stream(c, stream), a, pm, blocks,
              threads, phases, scope_dev, wave_mask_dev, op_off_dev, n_op_off, ops_dev, n_ops,
              block_map_dev, lds_words, (const uint16_t*)c->fsm_tab);
    return HR_OK;
}
