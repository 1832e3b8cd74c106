// Fixture for the structural assembly checks of tests/test_isa.py.  It is
// compiled to assembly on the host only and is never built into the library
// nor launched: it gives the checker one kernel with a work-group barrier
// inside a loop whose trip count depends on the lane (which must be flagged)
// and one with the barrier after such a loop (which must not be).
#include <hip/hip_runtime.h>

__global__ void fixture_barrier_in_lane_dependent_loop(int *p, int n)
{
    __shared__ int s[256];
    for (int i = threadIdx.x; i < n; i += 64) {
        s[threadIdx.x] = i;
        __syncthreads();
        p[i] = s[(threadIdx.x + 1) & 255];
    }
}

__global__ void fixture_barrier_after_lane_dependent_loop(int *p, int n)
{
    __shared__ int s[256];
    int acc = 0;
    for (int i = threadIdx.x; i < n; i += 64)
        acc += p[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    p[threadIdx.x] = s[(threadIdx.x + 1) & 255];
}
