// Example input of the source instrumenter: a histogram of n keys, one
// thread per key, with atomic increments, or with plain read-modify-write
// increments when `plain` is set (a race on every bin hit by two threads).
#include <hip/hip_runtime.h>

__global__ void histogram(const int* keys, int* bins, int n, int plain)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const int k = keys[i];
        if (plain) bins[k] += 1;
        else atomicAdd(&bins[k], 1);
    }
}
