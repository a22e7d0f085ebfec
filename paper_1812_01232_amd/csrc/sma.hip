// SMA, the local optimiser of Algorithm 1 (Section 6), as a library call:
// one block of 512 threads runs L-BFGS from each start (sma_core.h holds the
// objective, its gradient and the L-BFGS loop).
#include "sma_core.h"

namespace gosma {
namespace {

using namespace sma;

// One block per start: starts x0[n][6] (r, t); outputs x_out[n][6], f_out,
// g_out[n][6] (gradient at the result, may be NULL), it_out.
__global__ __launch_bounds__(kSmaThreads) void k_sma(DevMix mx, int64_t n, const uint32_t *__restrict__ pids,
                                                   const double *__restrict__ x0, int max_iters, int memory,
                                                   double gtol, double ftol, double *x_out, double *f_out,
                                                   double *g_out, int32_t *it_out)
{
    extern __shared__ float4 lds[];
    __shared__ SmaShared sh;
    __shared__ SmaState st;
    const int tid = threadIdx.x;
    for (int64_t s = blockIdx.x; s < n; s += gridDim.x) {
        const uint32_t pid = pids ? pids[s] : 0u;
        const bool bad_pid = pid >= (uint32_t)mx.n_prob;
        __syncthreads();
        if (tid == 0)
            for (int a = 0; a < 6; ++a) sh.x[a] = x0[6 * s + a];
        __syncthreads();
        double x[6], f, g[6];
        int it = -1;
        if (bad_pid) {
            for (int a = 0; a < 6; ++a) {
                x[a] = sh.x[a];
                g[a] = 0.0;
            }
            f = NAN;
        } else {
            const ProbDesc P = mx.prob[pid];
            float4 *base = mx.grec ? mx.grec + (int64_t)blockIdx.x * mx.grec_stride : lds;
            it = sma_run(mx, P, sh, st, sma_lds(base, P.M, P.N), max_iters, memory, gtol, ftol, x, f, g);
        }
        if (tid == 0) {
            for (int a = 0; a < 6; ++a) {
                x_out[6 * s + a] = x[a];
                if (g_out) g_out[6 * s + a] = g[a];
            }
            f_out[s] = f;
            it_out[s] = it;
        }
    }
}

}  // namespace

size_t sma_lds_bytes(int maxM, int maxN)
{
    return (size_t)maxM * (2 * sizeof(float4) + sizeof(float2) + sizeof(int)) +
           (size_t)maxN * (sizeof(float4) + sizeof(float2));
}

hipError_t launch_sma(const DevMix &mx, int maxM, int maxN, int64_t n, const uint32_t *pids, const double *x0,
                      int max_iters, int memory, double gtol, double ftol, double *x_out, double *f_out,
                      double *g_out, int32_t *it_out, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    // records in LDS, or (mixtures too large for it) in the global records, one slice per block
    const size_t lds = mx.grec ? 0 : sma_lds_bytes(maxM, maxN);
    if (!mx.grec) {
        hipError_t e = hipFuncSetAttribute((const void *)k_sma, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    const int64_t gmax = mx.grec ? mx.grec_blocks : 4096;
    const int grid = (int)(n < gmax ? n : gmax);
    hipLaunchKernelGGL(k_sma, dim3(grid), dim3(kSmaThreads), lds, stream, mx, n, pids, x0, max_iters, memory, gtol,
                       ftol, x_out, f_out, g_out, it_out);
    return hipGetLastError();
}

}  // namespace gosma
