// Small device helpers of the host runtime.
#include <hip/hip_runtime.h>

#include <algorithm>

namespace hybfs {

__global__ void zero_kernel(unsigned long long *p, long long words)
{
    const long long nt = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += nt) p[i] = 0ull;
}

hipError_t launch_zero(void *p, size_t bytes, hipStream_t s)
{
    const long long words = (long long)(bytes / 8);
    if (words <= 0) return hipSuccess;
    const long long blocks = std::min<long long>((words + 255) / 256, 1024);
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, s, (unsigned long long *)p, words);
    return hipGetLastError();
}

}  // namespace hybfs
