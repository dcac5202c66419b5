// Example input of the source instrumenter: the two-level reduction of
// tile_reduce.hip written with cooperative groups.  Each 8-lane tile
// (cg::tiled_partition<8>) sums its 16 input words in its own LDS segment,
// synchronizing with tile.sync(); lane 0 of each tile stores the tile's sum
// in its wave's slot array, and the wave (cg::tiled_partition<64>) sums
// the slots with wave.sync(); a block.sync() ends the reduction, then every
// lane writes its wave's total.  drop_tile / drop_wave remove the barrier
// after one tile step / one wave step (-1: none).  Blocks of 64 or 128
// threads.
#include <hip/hip_runtime.h>
#include <hip/hip_cooperative_groups.h>

namespace cg = cooperative_groups;

__global__ void cg_reduce(const int* in, int* out, int drop_tile, int drop_wave)
{
    __shared__ int s[320];
    cg::thread_block block = cg::this_thread_block();
    cg::thread_block_tile<8> tile = cg::tiled_partition<8>(block);
    cg::thread_block_tile<64> wave = cg::tiled_partition<64>(block);
    const int t = threadIdx.x, threads = blockDim.x;
    const int l = t & 7, g = t / 8, lw = t & 63;
    const int base = g * 16, T = 8;
    const int slots = 2 * threads + (t >> 6) * T;
    const int gb = blockIdx.x * threads * 2 + base;
    s[base + l] = in[gb + l];
    s[base + l + 8] = in[gb + l + 8];
    tile.sync();
    int step = 0;
    for (int h = 8; h > 0; h >>= 1, ++step) {
        if (l < h) s[base + l] = s[base + l] + s[base + l + h];
        if (step != drop_tile) tile.sync();
    }
    if (l == 0) s[slots + g % T] = s[base];
    wave.sync();
    step = 0;
    for (int h = T / 2; h > 0; h >>= 1, ++step) {
        if (lw < h) s[slots + lw] = s[slots + lw] + s[slots + lw + h];
        if (step != drop_wave) wave.sync();
    }
    block.sync();
    out[blockIdx.x * threads + t] = s[slots];
}
