// libchase_synth: device-side input generators (not part of the solver).
//
// The same counter-based definitions as the host generators: Philox4x32-10
// (Salmon et al., SC'11) keyed by the 64-bit seed, counter (i, j, stream, 0);
// two 53-bit uniforms per call; Box-Muller normals.  Device and host libm
// may differ in the last bit of log/sin/cos/exp.
//
//  synth_dk:     H = D + K (column-major, both triangles), entry (i, j) of
//                the lower triangle from counter (i, j, 1); D from (i, 0, 0).
//  synth_gauss:  complex Gaussian N x M (column-major), E|z|^2 = 1.
//  synth_copy:   plain device copy (reference kernel of known traffic).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace {

__device__ __forceinline__ void philox10(uint32_t c[4], uint32_t k0, uint32_t k1) {
    for (int rnd = 0; rnd < 10; ++rnd) {
        if (rnd) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        c[1] = (uint32_t)p1;
        c[3] = (uint32_t)p0;
        c[0] = n0;
        c[2] = n2;
    }
}

__device__ __forceinline__ double u53(uint32_t a, uint32_t b) {
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6) + 0.5) /
           9007199254740992.0;
}

__device__ __forceinline__ void uniforms(uint64_t i, uint64_t j, uint32_t stream,
                                         uint64_t seed, double &u1, double &u2) {
    uint32_t c[4] = {(uint32_t)i, (uint32_t)j, stream, 0u};
    philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    u1 = u53(c[0], c[1]);
    u2 = u53(c[2], c[3]);
}

__device__ __forceinline__ void normals(uint64_t i, uint64_t j, uint32_t stream,
                                        uint64_t seed, double &z0, double &z1) {
    double u1, u2;
    uniforms(i, j, stream, seed, u1, u2);
    const double r = sqrt(-2.0 * log(u1));
    const double t = 2.0 * M_PI * u2;
    z0 = r * cos(t);
    z1 = r * sin(t);
}

__global__ void k_dk(double2 *H, int64_t ld, int64_t N, uint64_t seed,
                     double std_, double decay, double lo, double hi) {
    const int64_t total = N * N;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t col = t / N, row = t - col * N;
        const int64_t i = row >= col ? row : col, j = row >= col ? col : row;
        double z0, z1;
        normals((uint64_t)i, (uint64_t)j, 1u, seed, z0, z1);
        double2 v;
        if (i == j) {
            double u1, u2;
            uniforms((uint64_t)i, 0, 0u, seed, u1, u2);
            v.x = std_ * z0 + (lo + (hi - lo) * u1);
            v.y = 0.0;
        } else {
            const double s = std_ * exp(-(double)(i - j) / decay) * sqrt(0.5);
            v.x = s * z0;
            v.y = s * z1;
            if (row < col) v.y = -v.y;   // upper triangle: conjugate
        }
        H[row + col * ld] = v;
    }
}

__global__ void k_gauss(double2 *G, int64_t ld, int64_t N, int64_t M,
                        uint64_t seed, uint32_t stream) {
    const int64_t total = N * M;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t col = t / N, row = t - col * N;
        double z0, z1;
        normals((uint64_t)row, (uint64_t)col, stream, seed, z0, z1);
        G[row + col * ld] = double2{z0 * sqrt(0.5), z1 * sqrt(0.5)};
    }
}

__global__ void k_copy(const double4 *__restrict__ src, double4 *__restrict__ dst,
                       int64_t n) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x)
        dst[t] = src[t];
}

int grid_for(int64_t total) {
    int64_t g = (total + 255) / 256;
    return (int)(g < 16384 ? (g > 0 ? g : 1) : 16384);
}

}  // namespace

extern "C" {

// Returns 0 or a hipError_t code.
int synth_dk(void *dH, int64_t ld, int64_t N, uint64_t seed, double std_,
             double decay, double lo, double hi, void *stream) {
    if (!dH || N < 1 || ld < N) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(k_dk, dim3(grid_for(N * N)), dim3(256), 0,
                       (hipStream_t)stream, (double2 *)dH, ld, N, seed, std_,
                       decay, lo, hi);
    return (int)hipGetLastError();
}

int synth_gauss(void *dG, int64_t ld, int64_t N, int64_t M, uint64_t seed,
                uint32_t stream_tag, void *stream) {
    if (!dG || N < 1 || M < 1 || ld < N) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gauss, dim3(grid_for(N * M)), dim3(256), 0,
                       (hipStream_t)stream, (double2 *)dG, ld, N, M, seed,
                       stream_tag);
    return (int)hipGetLastError();
}

// Copies `bytes` (a multiple of 32) from src to dst.
int synth_copy(const void *src, void *dst, int64_t bytes, void *stream) {
    if (!src || !dst || bytes < 0 || bytes % 32) return (int)hipErrorInvalidValue;
    const int64_t n = bytes / 32;
    hipLaunchKernelGGL(k_copy, dim3(grid_for(n)), dim3(256), 0,
                       (hipStream_t)stream, (const double4 *)src, (double4 *)dst, n);
    return (int)hipGetLastError();
}

}  // extern "C"
