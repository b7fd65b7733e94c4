// Device copies and the cross-block maximum of a domain cut into blocks on one GPU.
#include "fsa_impl.hpp"

namespace fsa {

namespace {

// Every entry a contiguous run of doubles; blockIdx.y picks the entry.
__global__ __launch_bounds__(256) void k_copy_list(const CopyEntry* __restrict__ list)
{
    const CopyEntry e = list[blockIdx.y];
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < e.count;
         i += (long long)gridDim.x * blockDim.x)
        e.dst[i] = e.src[i];
}

// The NaN-propagating maximum over nb blocks' wave-speed slots, written into each block's
// destination slot.
__global__ void k_amax_blocks(unsigned long long* const* __restrict__ in, unsigned long long* const* __restrict__ out,
                              int nb)
{
    const int d = threadIdx.x;
    if (d >= 3) return;
    unsigned long long v = 0ull;
    for (int b = 0; b < nb; ++b) v = max_bits(v, in[b][d]);
    for (int b = 0; b < nb; ++b) out[b][d] = v;
}

}  // namespace

int launch_copy_list(const CopyEntry* d_list, int n, long long max_count, hipStream_t s)
{
    if (n <= 0 || max_count <= 0) return 0;
    const long long want = (max_count + 255) / 256;
    const dim3 grid((unsigned)std::min<long long>(want, 1024), (unsigned)n);
    hipLaunchKernelGGL(k_copy_list, grid, dim3(256), 0, s, d_list);
    return (int)hipGetLastError();
}

int launch_amax_blocks(unsigned long long* const* d_in, unsigned long long* const* d_out, int nb, hipStream_t s)
{
    hipLaunchKernelGGL(k_amax_blocks, dim3(1), dim3(64), 0, s, d_in, d_out, nb);
    return (int)hipGetLastError();
}

}  // namespace fsa
