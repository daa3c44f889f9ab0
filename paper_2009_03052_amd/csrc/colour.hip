// Colourings (Sec. 2 and Sec. 3.5, "Biased coloring"): the biased law on the
// device and the probability that a vertex set receives a given colour set.
#include <cmath>

#include "device.hpp"

namespace {

// colour 0 with probability 1 - (k-1) L / 2^32, each colour in [1, k) with
// L / 2^32: the low 32 bits r of the first Philox output for key (seed,
// stream) and counter (v, 0, 1, 0) give colour 0 while r < 2^32 - (k-1) L,
// else 1 + (r - (2^32 - (k-1) L)) / L
__global__ void __launch_bounds__(256) k_color_biased(int64_t n, int k, uint32_t L, uint64_t seed, uint64_t stream,
                                                      uint8_t *out)
{
    const uint64_t t0 = (1ull << 32) - (uint64_t)(k - 1) * L;
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += step) {
        uint64_t c[4] = {(uint64_t)v, 0, 1, 0};
        philox4x64_10(c, seed, stream);
        const uint32_t r = (uint32_t)c[0];
        out[v] = r < t0 ? 0 : (uint8_t)(1u + (uint32_t)((r - t0) / L));
    }
}

// lambda in units of 2^-32; 0 when out of range for k
uint32_t lambda_units(int k, double lambda)
{
    if (!(lambda > 0) || k < 2) return 0;
    const double q = std::nearbyint(lambda * 4294967296.0);
    if (q < 1 || q > 4294967295.0 || q * (k - 1) > 4294967296.0) return 0;
    return (uint32_t)q;
}

}  // namespace

extern "C" scc_status scc_color_biased(int64_t n, int k, double lambda, uint64_t seed, uint64_t stream_id,
                                       uint8_t *colors, void *stream)
{
    if (k < 2 || k > SCC_KMAX) return set_error(SCC_EINVAL, "k = %d not in [2, 8]", k);
    if (n < 0) return set_error(SCC_EINVAL, "n < 0");
    const uint32_t L = lambda_units(k, lambda);
    if (!L) return set_error(SCC_EINVAL, "lambda = %g outside (0, 1/(k-1)] in units of 2^-32", lambda);
    if (n == 0) return SCC_OK;
    if (!colors) return set_error(SCC_EINVAL, "colors NULL");
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 256 * 64);
    hipLaunchKernelGGL(k_color_biased, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, n, k, L, seed,
                       stream_id, colors);
    HIP_TRY(hipGetLastError());
    return SCC_OK;
}

extern "C" double scc_colour_set_probability(int k, double lambda, int j, int has_zero)
{
    if (k < 1 || k > SCC_KMAX || j < 1 || j > k) return -1.0;
    double p = 1.0;
    for (int i = 2; i <= j; i++) p *= i;
    if (lambda <= 0) {
        for (int i = 0; i < j; i++) p /= k;   // uniform colours: j! / k^j
        return p;
    }
    const uint32_t L = lambda_units(k, lambda);
    if (!L) return -1.0;
    const double lam = (double)L / 4294967296.0;
    for (int i = 0; i < (has_zero ? j - 1 : j); i++) p *= lam;
    if (has_zero) p *= 1.0 - (double)(k - 1) * lam;
    return p;
}
