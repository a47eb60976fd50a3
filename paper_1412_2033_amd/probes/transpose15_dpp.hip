// Measurement probe (not part of the library): the exchange between the two
// radix-15 stages of a 225-point transform is a 15 x 15 transpose across the
// 15 (+1 spare) lanes that own the transform.  Here a 16 x 16 complex FP32
// transpose within each aligned 16-lane group, repeated REPS times in
// registers, two ways: through LDS (16 ds_write_b64 into a padded row of the
// lane, 16 ds_read_b64 of a column), as the transform kernels do, and with
// cross-lane moves only (a per-lane rotation by the lane index as a barrel
// shifter of selects, one DPP row rotation per register, the inverse
// rotation).  Each form is first checked against the transpose on the host.
//
//   hipcc --offload-arch=gfx950 -O3 -std=c++17 -Xclang -target-feature \
//       -Xclang -packed-fp32-ops paper_1412_2033_amd/probes/transpose15_dpp.hip \
//       -o /tmp/transpose15_dpp && /tmp/transpose15_dpp
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdlib>
#include <vector>

// rotate u left by (li mod 16): u'[k] = u[(k + li) mod 16], as four stages of
// bitwise selects (one v_bfi_b32 per element and stage)
__device__ __forceinline__ void rotl_lane(float *re, float *im, int li) {
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int s = 1 << b;
        const unsigned m = 0u - (unsigned)((li >> b) & 1);  // all ones: take the shifted element
        unsigned nr[16], ni[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const unsigned a0 = __float_as_uint(re[k]), a1 = __float_as_uint(re[(k + s) & 15]);
            const unsigned b0 = __float_as_uint(im[k]), b1 = __float_as_uint(im[(k + s) & 15]);
            nr[k] = (a1 & m) | (a0 & ~m);
            ni[k] = (b1 & m) | (b0 & ~m);
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            re[k] = __uint_as_float(nr[k]);
            im[k] = __uint_as_float(ni[k]);
            // keep the four stages apart (merged, they become one 16-way
            // select per element)
            asm volatile("" : "+v"(re[k]), "+v"(im[k]));
        }
    }
}

template <int K>
__device__ __forceinline__ float ror(float v) {
    // DPP row_ror:K (rotate within each row of 16 lanes)
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x120 + K, 0xF, 0xF, false));
}

template <int K>
__device__ __forceinline__ void ror_all(float *re, float *im) {
    if constexpr (K < 16) {
        re[K] = ror<K>(re[K]);
        im[K] = ror<K>(im[K]);
        ror_all<K + 1>(re, im);
    }
}

// lane i of a group holds row i (a[i][k] in register k); afterwards column i
__device__ __forceinline__ void transpose_dpp(float *re, float *im, int li) {
    rotl_lane(re, im, li);  // b[k] = a[i][(k + i) mod 16]
    ror_all<1>(re, im);     // register k from the lane k places below (row_ror:k)
    // c[k] = a[(i - k) mod 16][i]: reverse, then rotate right by i
    float r2[16], i2[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        r2[k] = re[(16 - k) & 15];
        i2[k] = im[(16 - k) & 15];
    }
    rotl_lane(r2, i2, (16 - li) & 15);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        re[k] = r2[k];
        im[k] = i2[k];
    }
}

__global__ __launch_bounds__(256) void tr_dpp(const float2 *X, float2 *Y, int reps) {
    const long t = blockIdx.x * 256L + threadIdx.x;
    const int li = threadIdx.x & 15;
    float re[16], im[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const float2 v = X[t * 16 + k];
        re[k] = v.x;
        im[k] = v.y;
    }
    for (int r = 0; r < reps; ++r) transpose_dpp(re, im, li);
#pragma unroll
    for (int k = 0; k < 16; ++k) Y[t * 16 + k] = make_float2(re[k], im[k]);
}

__global__ __launch_bounds__(256) void tr_lds(const float2 *X, float2 *Y, int reps) {
    __shared__ float2 buf[16][16 * 17];  // per 16-lane group: 16 rows of 17 (padded)
    const long t = blockIdx.x * 256L + threadIdx.x;
    const int li = threadIdx.x & 15, grp = threadIdx.x >> 4;
    float2 u[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) u[k] = X[t * 16 + k];
    float2 *B = buf[grp];
    for (int r = 0; r < reps; ++r) {
#pragma unroll
        for (int k = 0; k < 16; ++k) B[li * 17 + k] = u[k];
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int k = 0; k < 16; ++k) u[k] = B[k * 17 + li];
        __builtin_amdgcn_wave_barrier();
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) Y[t * 16 + k] = u[k];
}

#define CK(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) { printf("HIP error %s at %d\n", hipGetErrorString(e_), __LINE__); exit(1); } } while (0)

int main() {
    const int nblocks = 4096;
    const long nt = (long)nblocks * 256;
    std::vector<float2> hx(nt * 16), hy(nt * 16);
    for (long i = 0; i < nt * 16; ++i) hx[i] = make_float2((float)(i % 977), (float)(i % 631));
    float2 *dx, *dy;
    CK(hipMalloc(&dx, nt * 16 * sizeof(float2)));
    CK(hipMalloc(&dy, nt * 16 * sizeof(float2)));
    CK(hipMemcpy(dx, hx.data(), nt * 16 * sizeof(float2), hipMemcpyHostToDevice));
    const int reps = 64;
    for (int kind = 0; kind < 2; ++kind) {
        auto launch = [&](int rp) {
            if (kind == 0)
                hipLaunchKernelGGL(tr_lds, dim3(nblocks), dim3(256), 0, 0, dx, dy, rp);
            else
                hipLaunchKernelGGL(tr_dpp, dim3(nblocks), dim3(256), 0, 0, dx, dy, rp);
            CK(hipGetLastError());
        };
        launch(1);
        CK(hipDeviceSynchronize());
        CK(hipMemcpy(hy.data(), dy, nt * 16 * sizeof(float2), hipMemcpyDeviceToHost));
        long bad = 0;
        for (long t = 0; t < nt; ++t) {
            const long g0 = t - (t & 15);  // first thread of the group
            const int i = (int)(t & 15);
            for (int k = 0; k < 16; ++k) {
                const float2 want = hx[(g0 + k) * 16 + i];  // a[k][i]
                const float2 got = hy[t * 16 + k];
                if (got.x != want.x || got.y != want.y) ++bad;
            }
        }
        hipEvent_t e0, e1;
        CK(hipEventCreate(&e0));
        CK(hipEventCreate(&e1));
        launch(reps);
        CK(hipEventRecord(e0, 0));
        const int runs = 10;
        for (int i = 0; i < runs; ++i) launch(reps);
        CK(hipEventRecord(e1, 0));
        CK(hipEventSynchronize(e1));
        float ms = 0;
        CK(hipEventElapsedTime(&ms, e0, e1));
        const double trs = (double)(nt / 16) * reps * runs;  // 16 x 16 transposes
        printf("%s: %ld wrong elements after one transpose; %d transposes per group: %.3f ms per launch, %.2f G transposes/s\n",
               kind == 0 ? "LDS" : "DPP+selects", bad, reps, ms / runs, trs / (ms * 1e-3) / 1e9);
        fflush(stdout);
    }
    return 0;
}
