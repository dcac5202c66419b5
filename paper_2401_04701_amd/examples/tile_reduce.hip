// Example input of the source instrumenter: a two-level reduction with tiles
// nested in waves.  Each tile of `tile` lanes (a power of two from 2 to 32)
// sums its 2 * tile input words in its own LDS segment by halving steps,
// synchronizing only its own lanes with __syncwarp(mask of the tile); lane
// 0 of each tile then stores the tile's sum in its wave's slot array, and
// the wave sums the slots by halving steps with whole-wave __syncwarp().
// Every lane writes its wave's total.  drop_tile / drop_wave remove the
// barrier after one tile step / one wave step (-1: none).  Blocks of 64 or
// 128 threads.
#include <hip/hip_runtime.h>

__global__ void tile_reduce(const int* in, int* out, int tile, int drop_tile, int drop_wave)
{
    __shared__ int s[320];
    const int t = threadIdx.x, threads = blockDim.x;
    const int lane = t & 63, l = t & (tile - 1), g = t / tile;
    const int n = 2 * tile, base = g * n, T = 64 / tile;
    const int slots = 2 * threads + (t >> 6) * T, lw = lane;
    const unsigned long long mine = ((1ull << tile) - 1ull) << (lane & ~(tile - 1));
    const int gb = blockIdx.x * threads * 2 + base;
    s[base + l] = in[gb + l];
    s[base + l + tile] = in[gb + l + tile];
    __syncwarp(mine);
    int step = 0;
    for (int h = tile; h > 0; h >>= 1, ++step) {
        if (l < h) s[base + l] = s[base + l] + s[base + l + h];
        if (step != drop_tile) __syncwarp(mine);
    }
    if (l == 0) s[slots + g % T] = s[base];
    __syncwarp();
    step = 0;
    for (int h = T / 2; h > 0; h >>= 1, ++step) {
        if (lw < h) s[slots + lw] = s[slots + lw] + s[slots + lw + h];
        if (step != drop_wave) __syncwarp();
    }
    out[blockIdx.x * threads + t] = s[slots];
}
