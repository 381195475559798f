// Probe block of Alg. 3: independent N(0,1) vectors from a counter-based
// generator, so any entry can be regenerated from (seed, row, column) alone.
//
// Philox4x64-10 (Salmon, Moraes, Dror & Shaw, SC'11): key (seed, 0), counter
// (row / 4, column, 0, 0); the four 64-bit words give uniforms
// u = ((x >> 11) + 1) 2^-53 in (0, 1] and Box-Muller pairs
// (sqrt(-2 ln u0) cos(2 pi u1), sqrt(-2 ln u0) sin(2 pi u1)) for rows 4q, 4q+1 and
// the same from (u2, u3) for rows 4q+2, 4q+3, all in float64, then rounded to
// float32 and (bfloat16 storage) to bfloat16.
#include <cmath>

#include "common.h"

namespace {

struct u64x4 {
    uint64_t v[4];
};

// Full 128-bit product of a 64-bit word and the constant M = (mh, ml), from the four
// 32 x 32 -> 64 partial products, each with the carry-in folded into its addend (so
// each is one multiply-add on the vector unit, and the low word reuses them).
__device__ __forceinline__ void mul_128(uint64_t x, uint32_t mh, uint32_t ml, uint64_t& hi, uint64_t& lo) {
    const uint32_t xl = (uint32_t)x, xh = (uint32_t)(x >> 32);
    const uint64_t p00 = (uint64_t)xl * ml;
    const uint64_t t = (uint64_t)xl * mh + (p00 >> 32);          // < 2^64
    const uint64_t u = (uint64_t)xh * ml + (uint32_t)t;          // < 2^64
    lo = (u << 32) | (uint32_t)p00;
    hi = (uint64_t)xh * mh + ((t >> 32) + (u >> 32));            // the high word of x M
}

__device__ __forceinline__ u64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                                               uint64_t k1) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t hi0, lo0, hi1, lo1;
        mul_128(c0, (uint32_t)(M0 >> 32), (uint32_t)M0, hi0, lo0);
        mul_128(c2, (uint32_t)(M1 >> 32), (uint32_t)M1, hi1, lo1);
        const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    u64x4 r;
    r.v[0] = c0;
    r.v[1] = c1;
    r.v[2] = c2;
    r.v[3] = c3;
    return r;
}

__device__ __forceinline__ double unit_open0(uint64_t x) { return (double)((x >> 11) + 1) * 0x1.0p-53; }

template <typename T>
struct alignas(4 * sizeof(T)) quad_of {
    T v[4];
};

// One thread per group of four rows of one column; column j = blockIdx.y (no
// division of a flat index).  `vec`: n % 4 == 0 and X is aligned, so every group of
// four rows is whole and one store writes it.
template <typename T>
__global__ void probes_kernel(int64_t n, uint64_t seed, T* __restrict__ X, int vec) {
    const int64_t quads = (n + 3) / 4;
    const int j = blockIdx.y;
    T* col = X + (int64_t)j * n;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < quads; q += (int64_t)gridDim.x * blockDim.x) {
        const u64x4 x = philox4x64_10((uint64_t)q, (uint64_t)j, 0, 0, seed, 0);
        double z[4];
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            const double rad = sqrt(-2.0 * log(unit_open0(x.v[2 * half])));
            // angle 2 pi u as pi (2u): 2u is exact and lies in (0, 2], so sincospi needs
            // no range reduction beyond its own
            double sn, cs;
            sincospi(2.0 * unit_open0(x.v[2 * half + 1]), &sn, &cs);
            z[2 * half] = rad * cs;
            z[2 * half + 1] = rad * sn;
        }
        if (vec) {
            quad_of<T> w;
#pragma unroll
            for (int t = 0; t < 4; ++t) w.v[t] = from_f64<T>(z[t]);
            *(quad_of<T>*)(col + 4 * q) = w;
        } else {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int64_t r = 4 * q + t;
                if (r < n) col[r] = from_f64<T>(z[t]);
            }
        }
    }
}

}  // namespace

int probes_launch(bfgsuq_ctx* h, uint64_t seed, int32_t c, void* X, hipStream_t stream) {
    const int64_t quads = (h->n + 3) / 4;
    // columns on grid.y; along a column enough workgroups that c of them fill the GPU
    const int gx = (int)std::min<int64_t>(std::max<int64_t>(1, 16384 / c), (quads + 255) / 256);
    const dim3 grid(gx, c);
    const size_t tsz = dtype_size(h->storage);
    const int vec = h->n % 4 == 0 && (uintptr_t)X % (4 * tsz) == 0;
    switch (h->storage) {
        case BFGS_F64:
            hipLaunchKernelGGL(probes_kernel<double>, grid, dim3(256), 0, stream, h->n, seed, (double*)X, vec);
            break;
        case BFGS_F32:
            hipLaunchKernelGGL(probes_kernel<float>, grid, dim3(256), 0, stream, h->n, seed, (float*)X, vec);
            break;
        case BFGS_BF16:
            hipLaunchKernelGGL(probes_kernel<bf16_t>, grid, dim3(256), 0, stream, h->n, seed, (bf16_t*)X, vec);
            break;
    }
    return hipGetLastError() == hipSuccess ? BFGS_OK : BFGS_ERR_HIP;
}

int probes_run(bfgsuq_ctx* h, uint64_t seed, int32_t ncols, void* X) {
    return probes_launch(h, seed, ncols, X, h->stream);
}
