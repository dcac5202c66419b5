// Example input of the source instrumenter: a 3-point stencil over n floats
// in blocks of 256 threads that stage a 258-word LDS tile; the block
// `seeded_block` also writes the first cell owned by the next block (a
// seeded cross-block race).
#include <hip/hip_runtime.h>

__global__ void stencil3(const float* u, float* v, int n, int seeded_block)
{
    __shared__ float tile[258];
    const int l = threadIdx.x;
    const int g = blockIdx.x * 256 + l;
    if (g < n) tile[l + 1] = u[g];
    if (l == 0 && g > 0) tile[0] = u[g - 1];
    if (l == 255 && g + 1 < n) tile[257] = u[g + 1];
    __syncthreads();
    if (g < n) {
        const float c = tile[l + 1];
        const float left = g > 0 ? tile[l] : c;
        const float right = g + 1 < n ? tile[l + 2] : c;
        v[g] = (left + c + right) / 3.0f;
        if ((int)blockIdx.x == seeded_block && l == 255 && g + 1 < n) v[g + 1] = c;
    }
}
