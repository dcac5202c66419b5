// Instrumented workloads: a one-block LDS tree reduction, a 5-point Jacobi
// sweep with LDS halo staging, label propagation over a CSR graph, and an
// interpreter of access programs.  Each kernel is a template on CHECK so the
// plain (uninstrumented) kernel is the same code with the hooks compiled out.
#include <hip/hip_runtime.h>

#include "hr.h"
#include "hr_device.h"
#include "hr_internal.h"

namespace {

bool region_ok(hr_ctx c, uint32_t r, const void* data, size_t min_elems)
{
    return r < c->n_reg && c->reg[r].data == data && c->reg[r].elems >= min_elems;
}

// ---------------------------------------------------------------- reduce
template <bool CHECK>
__global__ __launch_bounds__(256) void k_reduce(hr_kargs a, uint32_t r_in, uint32_t r_out,
                                                const int32_t* __restrict__ in,
                                                int32_t* __restrict__ out, int32_t drop)
{
    __shared__ int32_t s[512];
    __shared__ uint32_t sh[512];
    const uint32_t t = threadIdx.x;
    hr_thread th{};
    if constexpr (CHECK) {
        th = hr_thread_make(a, blockIdx.x, t);
        sh[t] = 0;
        sh[t + 256] = 0;
        __syncthreads();
    }
    s[t] = in[t];
    if constexpr (CHECK) {
        hr_access<HR_READ>(a, th, r_in, t);
        hr_access_lds<HR_WRITE>(a, th, sh, 512, 0, t);
    }
    s[t + 256] = in[t + 256];
    if constexpr (CHECK) {
        hr_access<HR_READ>(a, th, r_in, t + 256);
        hr_access_lds<HR_WRITE>(a, th, sh, 512, 0, t + 256);
    }
    for (int32_t step = 0; step < 9; ++step) {
        const uint32_t h = 256u >> step;
        if (t < h) {
            const int32_t x = s[t];
            if constexpr (CHECK) hr_access_lds<HR_READ>(a, th, sh, 512, 0, t);
            const int32_t y = s[t + h];
            if constexpr (CHECK) hr_access_lds<HR_READ>(a, th, sh, 512, 0, t + h);
            s[t] = x + y;
            if constexpr (CHECK) hr_access_lds<HR_WRITE>(a, th, sh, 512, 0, t);
        }
        if (step != drop) {
            if constexpr (CHECK) hr_barrier_block(a, th);
            else __syncthreads();
        }
    }
    const int32_t r = s[0];
    if constexpr (CHECK) hr_access_lds<HR_READ>(a, th, sh, 512, 0, 0);
    out[t] = r;
    if constexpr (CHECK) hr_access<HR_WRITE>(a, th, r_out, t);
}

// ---------------------------------------------------------------- jacobi
constexpr uint32_t TILE = 18;
constexpr uint32_t TILE_WORDS = TILE * TILE;

template <bool CHECK>
__global__ __launch_bounds__(256) void k_jacobi(hr_kargs a, uint32_t r_old, uint32_t r_new,
                                                const float* __restrict__ uo,
                                                float* __restrict__ un, uint32_t ny, uint32_t nx,
                                                const int32_t* __restrict__ seeds)
{
    __shared__ float tile[TILE_WORDS];
    __shared__ uint32_t tsh[TILE_WORDS];
    const uint32_t t = threadIdx.x, tx = t & 15u, ty = t >> 4;
    const uint32_t b = blockIdx.y * gridDim.x + blockIdx.x;
    const uint32_t gx = blockIdx.x * 16u + tx, gy = blockIdx.y * 16u + ty;
    const bool inside = gx < nx && gy < ny;
    hr_thread th{};
    if constexpr (CHECK) {
        th = hr_thread_make(a, b, t);
        tsh[t] = 0;
        if (t < TILE_WORDS - 256) tsh[t + 256] = 0;
        __syncthreads();
    }
    const size_t g = (size_t)gy * nx + gx;
    const uint32_t cl = (ty + 1) * TILE + tx + 1;
    if (inside) {
        tile[cl] = uo[g];
        if constexpr (CHECK) {
            hr_access<HR_READ>(a, th, r_old, g);
            hr_access_lds<HR_WRITE>(a, th, tsh, TILE_WORDS, 0, cl);
        }
        if (ty == 0 && gy > 0) {
            tile[tx + 1] = uo[g - nx];
            if constexpr (CHECK) {
                hr_access<HR_READ>(a, th, r_old, g - nx);
                hr_access_lds<HR_WRITE>(a, th, tsh, TILE_WORDS, 0, tx + 1);
            }
        }
        if (ty == 15 && gy + 1 < ny) {
            tile[17 * TILE + tx + 1] = uo[g + nx];
            if constexpr (CHECK) {
                hr_access<HR_READ>(a, th, r_old, g + nx);
                hr_access_lds<HR_WRITE>(a, th, tsh, TILE_WORDS, 0, 17 * TILE + tx + 1);
            }
        }
        if (tx == 0 && gx > 0) {
            tile[(ty + 1) * TILE] = uo[g - 1];
            if constexpr (CHECK) {
                hr_access<HR_READ>(a, th, r_old, g - 1);
                hr_access_lds<HR_WRITE>(a, th, tsh, TILE_WORDS, 0, (ty + 1) * TILE);
            }
        }
        if (tx == 15 && gx + 1 < nx) {
            tile[(ty + 1) * TILE + 17] = uo[g + 1];
            if constexpr (CHECK) {
                hr_access<HR_READ>(a, th, r_old, g + 1);
                hr_access_lds<HR_WRITE>(a, th, tsh, TILE_WORDS, 0, (ty + 1) * TILE + 17);
            }
        }
    }
    if constexpr (CHECK) hr_barrier_block(a, th);
    else __syncthreads();
    if (inside) {
        const float c = tile[cl];
        if constexpr (CHECK) hr_access_lds<HR_READ>(a, th, tsh, TILE_WORDS, 0, cl);
        float vn = c, vs = c, vw = c, ve = c;
        if (gy > 0) {
            vn = tile[cl - TILE];
            if constexpr (CHECK) hr_access_lds<HR_READ>(a, th, tsh, TILE_WORDS, 0, cl - TILE);
        }
        if (gy + 1 < ny) {
            vs = tile[cl + TILE];
            if constexpr (CHECK) hr_access_lds<HR_READ>(a, th, tsh, TILE_WORDS, 0, cl + TILE);
        }
        if (gx > 0) {
            vw = tile[cl - 1];
            if constexpr (CHECK) hr_access_lds<HR_READ>(a, th, tsh, TILE_WORDS, 0, cl - 1);
        }
        if (gx + 1 < nx) {
            ve = tile[cl + 1];
            if constexpr (CHECK) hr_access_lds<HR_READ>(a, th, tsh, TILE_WORDS, 0, cl + 1);
        }
        const float r = 0.2f * (c + vn + vs + vw + ve);
        un[g] = r;
        if constexpr (CHECK) hr_access<HR_WRITE>(a, th, r_new, g);
        if (seeds) {
            const int32_t sd = seeds[b];
            if (sd >= 0) {
                const uint32_t side = (uint32_t)sd >> 8, off = (uint32_t)sd & 255u;
                int64_t tgt = -1;
                if (side == 0 && ty == 0 && tx == off && gy > 0) tgt = (int64_t)g - nx;
                else if (side == 1 && ty == 15 && tx == off && gy + 1 < ny) tgt = (int64_t)g + nx;
                else if (side == 2 && tx == 0 && ty == off && gx > 0) tgt = (int64_t)g - 1;
                else if (side == 3 && tx == 15 && ty == off && gx + 1 < nx) tgt = (int64_t)g + 1;
                if (tgt >= 0) {
                    un[tgt] = r;
                    if constexpr (CHECK) hr_access<HR_WRITE>(a, th, r_new, (uint64_t)tgt);
                }
            }
        }
    }
}

// ------------------------------------------------------------- labelprop
template <bool CHECK>
__global__ __launch_bounds__(1024) void k_labelprop(hr_kargs a, uint32_t r_label,
                                                    uint32_t r_rp, uint32_t r_col,
                                                    int32_t* __restrict__ label,
                                                    const int32_t* __restrict__ rp,
                                                    const int32_t* __restrict__ col,
                                                    const uint8_t* __restrict__ mask, uint32_t n)
{
    const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    hr_thread th{};
    if constexpr (CHECK) th = hr_thread_make(a, blockIdx.x, threadIdx.x);
    const int32_t l = __hip_atomic_load(label + v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if constexpr (CHECK) hr_access<HR_ATOMIC>(a, th, r_label, v);
    const int32_t e0 = rp[v], e1 = rp[v + 1];
    if constexpr (CHECK) {
        if (r_rp != UINT32_MAX) {
            hr_access<HR_READ>(a, th, r_rp, v);
            hr_access<HR_READ>(a, th, r_rp, v + 1);
        }
    }
    for (int32_t e = e0; e < e1; ++e) {
        const uint32_t u = (uint32_t)col[e];
        if constexpr (CHECK) {
            if (r_col != UINT32_MAX) hr_access<HR_READ>(a, th, r_col, (uint64_t)e);
        }
        if (u >= n) continue;
        if (mask[e]) {
            const int32_t r = label[u];
            if constexpr (CHECK) hr_access<HR_READ>(a, th, r_label, u);
            label[u] = r < l ? r : l;
            if constexpr (CHECK) hr_access<HR_WRITE>(a, th, r_label, u);
        } else {
            atomicMin(label + u, l);
            if constexpr (CHECK) hr_access<HR_ATOMIC>(a, th, r_label, u);
        }
    }
}

// ----------------------------------------------------------- interpreter
struct prog_map {
    uint32_t r[8];
};

__global__ __launch_bounds__(1024) void k_program(hr_kargs a, prog_map pm, uint32_t blocks,
                                                  uint32_t threads, uint32_t phases,
                                                  const uint8_t* __restrict__ scope,
                                                  const uint64_t* __restrict__ wmask,
                                                  const int32_t* __restrict__ op_off,
                                                  size_t n_op_off, const uint32_t* __restrict__ ops,
                                                  size_t n_ops, const uint32_t* __restrict__ bmap,
                                                  uint32_t lds_words)
{
    extern __shared__ uint32_t smem[];
    uint32_t* ldata = smem;
    uint32_t* lsh = smem + lds_words;
    const uint32_t b = bmap ? bmap[blockIdx.x] : blockIdx.x;
    if (b >= blocks) return;                      // uniform over the block
    const uint32_t t = threadIdx.x;
    hr_thread th = hr_thread_make(a, b, t);
    for (uint32_t i = t; i < lds_words; i += blockDim.x) {
        ldata[i] = 0;
        lsh[i] = 0;
    }
    __syncthreads();
    const uint32_t w = t >> 6;
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
            if (kind > 2) {
                hr_set_flag(a, HR_DEVF_RANGE);
                continue;
            }
            if ((op >> 29) & 1u) {
                if (idx >= lds_words) {
                    hr_set_flag(a, HR_DEVF_RANGE);
                    continue;
                }
                if (kind == 0) (void)*(volatile uint32_t*)(ldata + idx);
                else if (kind == 1) ldata[idx] = t + 1;
                else atomicAdd(ldata + idx, 1u);
                hr_access_lds_k(a, th, kind, lsh, lds_words, 0, idx);
            } else {
                const uint32_t r = pm.r[reg];
                if (r >= HR_MAX_REGIONS || idx >= a.n_elems[r]) {
                    hr_set_flag(a, HR_DEVF_RANGE);
                    continue;
                }
                uint32_t* d = (uint32_t*)a.data[r];
                if (kind == 0) (void)*(volatile uint32_t*)(d + idx);
                else if (kind == 1) d[idx] = t + 1;
                else atomicAdd(d + idx, 1u);
                hr_access_k(a, th, kind, r, idx);
            }
        }
        const uint8_t sc = scope[p];
        if (sc == 2) hr_barrier_block(a, th);
        else if (sc == 1 && w < 64 && ((wmask[p] >> w) & 1ull)) hr_barrier_wave(a, th);
    }
}

}  // namespace

// ======================================================================
extern "C" hr_status hr_reduce_check(hr_ctx c, uint32_t r_in, uint32_t r_out, const int32_t* in_dev,
                                     int32_t* out_dev, int32_t drop, void* stream)
{
    if (!c || !region_ok(c, r_in, in_dev, 512) || !region_ok(c, r_out, out_dev, 256))
        return HR_E_INVAL;
    hr_kargs a;
    hr_fill_args(c, &a);
    HR_LAUNCH(k_reduce<true>, dim3(1), dim3(256), 0, hr_stream(c, stream), a, r_in, r_out,
                       in_dev, out_dev, drop);
    return HR_OK;
}

extern "C" hr_status hr_reduce_plain(const int32_t* in_dev, int32_t* out_dev, int32_t drop,
                                     void* stream)
{
    if (!in_dev || !out_dev) return HR_E_INVAL;
    hr_kargs a{};
    HR_LAUNCH(k_reduce<false>, dim3(1), dim3(256), 0, (hipStream_t)stream, a, 0u, 0u,
                       in_dev, out_dev, drop);
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
    if (!c || !jacobi_shape_ok(ny, nx)) return HR_E_INVAL;
    const size_t cells = (size_t)ny * nx;
    if (!region_ok(c, r_old, u_old_dev, cells) || !region_ok(c, r_new, u_new_dev, cells))
        return HR_E_INVAL;
    hr_kargs a;
    hr_fill_args(c, &a);
    const dim3 grid((nx + 15) / 16, (ny + 15) / 16);
    HR_LAUNCH(k_jacobi<true>, grid, dim3(256), 0, hr_stream(c, stream), a, r_old, r_new,
                       u_old_dev, u_new_dev, ny, nx, seed_dev);
    return HR_OK;
}

extern "C" hr_status hr_jacobi_plain(const float* u_old_dev, float* u_new_dev, uint32_t ny,
                                     uint32_t nx, const int32_t* seed_dev, void* stream)
{
    if (!u_old_dev || !u_new_dev || !jacobi_shape_ok(ny, nx)) return HR_E_INVAL;
    hr_kargs a{};
    const dim3 grid((nx + 15) / 16, (ny + 15) / 16);
    HR_LAUNCH(k_jacobi<false>, grid, dim3(256), 0, (hipStream_t)stream, a, 0u, 0u,
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
    if (!c || !labelprop_shape_ok(n, tpb) || !region_ok(c, r_label, label_dev, n))
        return HR_E_INVAL;
    if (r_row_ptr != UINT32_MAX && !region_ok(c, r_row_ptr, row_ptr_dev, (size_t)n + 1))
        return HR_E_INVAL;
    if (r_col != UINT32_MAX && (r_col >= c->n_reg || c->reg[r_col].data != col_dev))
        return HR_E_INVAL;
    hr_kargs a;
    hr_fill_args(c, &a);
    HR_LAUNCH(k_labelprop<true>, dim3((n + tpb - 1) / tpb), dim3(tpb), 0,
                       hr_stream(c, stream), a, r_label, r_row_ptr, r_col, label_dev, row_ptr_dev,
                       col_dev, mask_dev, n);
    return HR_OK;
}

extern "C" hr_status hr_labelprop_plain(int32_t* label_dev, const int32_t* row_ptr_dev,
                                        const int32_t* col_dev, const uint8_t* mask_dev, uint32_t n,
                                        uint32_t tpb, void* stream)
{
    if (!label_dev || !row_ptr_dev || !col_dev || !mask_dev || !labelprop_shape_ok(n, tpb))
        return HR_E_INVAL;
    hr_kargs a{};
    HR_LAUNCH(k_labelprop<false>, dim3((n + tpb - 1) / tpb), dim3(tpb), 0,
                       (hipStream_t)stream, a, 0u, UINT32_MAX, UINT32_MAX, label_dev, row_ptr_dev,
                       col_dev, mask_dev, n);
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
        if (regions_host[i] >= c->n_reg) return HR_E_INVAL;
        pm.r[i] = regions_host[i];
    }
    hr_kargs a;
    hr_fill_args(c, &a);
    const size_t lds_bytes = (size_t)lds_words * 2 * sizeof(uint32_t);
    HR_LAUNCH(k_program, dim3(blocks), dim3(threads), lds_bytes, hr_stream(c, stream), a,
                       pm, blocks, threads, phases, scope_dev, wave_mask_dev, op_off_dev, n_op_off,
                       ops_dev, n_ops, block_map_dev, lds_words);
    return HR_OK;
}
