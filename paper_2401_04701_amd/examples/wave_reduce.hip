// Example input of the source instrumenter: each wave of a 256-thread block
// sums 128 input words in its own LDS segment by halving steps, with a
// wave-scope barrier (__syncwarp) after each step; `drop` removes the
// barrier after one step (a race inside every wave).
#include <hip/hip_runtime.h>

__global__ void wave_reduce(const int* in, int* out, int drop)
{
    __shared__ int s[512];
    const int t = threadIdx.x, l = t & 63, base = (t >> 6) * 128;
    const int g = blockIdx.x * 512 + base;
    s[base + l] = in[g + l];
    s[base + l + 64] = in[g + l + 64];
    int step = 0;
    for (int h = 64; h > 0; h >>= 1, ++step) {
        if (l < h) s[base + l] = s[base + l] + s[base + l + h];
        if (step != drop) __syncwarp();
    }
    out[blockIdx.x * 256 + t] = s[base];
}
