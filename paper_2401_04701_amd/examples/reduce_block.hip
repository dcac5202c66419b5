// Example input of the source instrumenter: a one-block tree reduction in
// LDS (512 int32 words, 256 threads) with a block barrier after each of its
// 9 halving steps, except the step named by `drop` (a seeded race).
#include <hip/hip_runtime.h>

__global__ void reduce_block(const int* in, int* out, int drop)
{
    __shared__ int a[512];
    const unsigned t = threadIdx.x;
    a[t] = in[t];
    a[t + 256] = in[t + 256];
    for (int s = 0; s < 9; ++s) {
        const unsigned h = 256u >> s;
        if (t < h) a[t] += a[t + h];
        if (s != drop) __syncthreads();
    }
    out[t] = a[0];
}
