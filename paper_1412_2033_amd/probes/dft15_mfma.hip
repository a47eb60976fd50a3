// Measurement probe (not part of the library): 15-point DFTs, the radix-15
// butterfly of the transform kernels (Good-Thomas 3 x 5) against the same DFT
// as a matrix product on the matrix cores (the 15 x 15 DFT matrix zero-padded
// to 16 x 16, four real products of v_mfma_f32_16x16x4f32 /
// v_mfma_f64_16x16x4f64 per complex product), FP32 and FP64.  Both keep their
// vectors in registers and apply REPS dependent DFTs, so the figures are the
// arithmetic throughput alone (a real stage adds the LDS exchanges and the
// twiddles; the matrix-core form would add moves into its operand layout).
// Each form is first checked against a direct long-double DFT.
//
//   hipcc --offload-arch=gfx950 -O3 -std=c++17 -Xclang -target-feature \
//       -Xclang -packed-fp32-ops -I include -I paper_1412_2033_amd/csrc \
//       paper_1412_2033_amd/probes/dft15_mfma.hip -o /tmp/dft15_mfma && /tmp/dft15_mfma
#include "fftgal_kernels.hip"
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <vector>
#include <complex>

using fftgal::Vt;

template <typename T>
__global__ __launch_bounds__(256) void bfly_kernel(const Vt<T> *X, Vt<T> *Y, int reps) {
    const long v = blockIdx.x * 256L + threadIdx.x;
    Vt<T> u[15];
#pragma unroll
    for (int q = 0; q < 15; ++q) u[q] = X[v * 16 + q];
    for (int r = 0; r < reps; ++r) fftgal::dftn<T, 15>(u, T(1));
#pragma unroll
    for (int q = 0; q < 15; ++q) Y[v * 16 + q] = u[q];
}

template <typename T> struct MV;
template <> struct MV<float> { typedef float __attribute__((ext_vector_type(4))) v4; };
template <> struct MV<double> { typedef double __attribute__((ext_vector_type(4))) v4; };

template <typename T>
__device__ __forceinline__ typename MV<T>::v4 mfma(T a, T b, typename MV<T>::v4 c) {
    if constexpr (sizeof(T) == 4)
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// lane l = c + 16 g holds, in result register i, row 4g + i of column c
// (FP32) or row g + 4i (FP64; measured); k-step s takes as B operand
// register s (row rm(g, s)) and as A operand F[c][rm(g, s)], so that the
// result is the B layout of the next product.
template <typename T, int TILES>
__global__ __launch_bounds__(256) void mfma_kernel(const Vt<T> *X, Vt<T> *Y, const T *Fr, const T *Fi, int reps) {
    using v4 = typename MV<T>::v4;
    const int lane = threadIdx.x & 63;
    const long wave = (blockIdx.x * 256L + threadIdx.x) >> 6;
    const int g = lane >> 4, c = lane & 15;
    auto rm = [&](int i) { return sizeof(T) == 4 ? 4 * g + i : g + 4 * i; };
    T ar[4], ai[4], nai[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        ar[s] = Fr[c * 16 + rm(s)];
        ai[s] = Fi[c * 16 + rm(s)];
        nai[s] = -ai[s];
    }
    v4 xr[TILES], xi[TILES];
#pragma unroll
    for (int t = 0; t < TILES; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = rm(i);
            const long vec = (wave * TILES + t) * 16 + c;
            const Vt<T> v = row < 15 ? X[vec * 16 + row] : Vt<T>{T(0), T(0)};
            xr[t][i] = v.x;
            xi[t][i] = v.y;
        }
    for (int r = 0; r < reps; ++r) {
        v4 yr[TILES], yi[TILES];
#pragma unroll
        for (int t = 0; t < TILES; ++t) {
            yr[t] = v4{T(0), T(0), T(0), T(0)};
            yi[t] = v4{T(0), T(0), T(0), T(0)};
        }
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int t = 0; t < TILES; ++t) {
                yr[t] = mfma<T>(ar[s], xr[t][s], yr[t]);
                yr[t] = mfma<T>(nai[s], xi[t][s], yr[t]);
                yi[t] = mfma<T>(ar[s], xi[t][s], yi[t]);
                yi[t] = mfma<T>(ai[s], xr[t][s], yi[t]);
            }
#pragma unroll
        for (int t = 0; t < TILES; ++t) {
            xr[t] = yr[t];
            xi[t] = yi[t];
        }
    }
#pragma unroll
    for (int t = 0; t < TILES; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = rm(i);
            const long vec = (wave * TILES + t) * 16 + c;
            if (row < 15) Y[vec * 16 + row] = Vt<T>{xr[t][i], xi[t][i]};
        }
}

#define CK(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) { printf("HIP error %s at %d\n", hipGetErrorString(e_), __LINE__); exit(1); } } while (0)

template <typename T>
void run(const char *name, int nblocks, int reps_time) {
    const long nvec = (long)nblocks * 256;
    std::vector<Vt<T>> hx(nvec * 16);
    srand(7);
    for (auto &v : hx) {
        v.x = T((rand() / (double)RAND_MAX - 0.5) * 1e-20);
        v.y = T((rand() / (double)RAND_MAX - 0.5) * 1e-20);
    }
    std::vector<T> fr(256, T(0)), fi(256, T(0));
    for (int m = 0; m < 15; ++m)
        for (int n = 0; n < 15; ++n) {
            const long double a = 2.0L * 3.141592653589793238462643383279502884L * ((m * n) % 15) / 15.0L;
            fr[m * 16 + n] = T(cosl(a));
            fi[m * 16 + n] = T(sinl(a));
        }
    Vt<T> *dx, *dy;
    T *dfr, *dfi;
    CK(hipMalloc(&dx, nvec * 16 * sizeof(Vt<T>)));
    CK(hipMalloc(&dy, nvec * 16 * sizeof(Vt<T>)));
    CK(hipMalloc(&dfr, 256 * sizeof(T)));
    CK(hipMalloc(&dfi, 256 * sizeof(T)));
    CK(hipMemcpy(dx, hx.data(), nvec * 16 * sizeof(Vt<T>), hipMemcpyHostToDevice));
    CK(hipMemcpy(dfr, fr.data(), 256 * sizeof(T), hipMemcpyHostToDevice));
    CK(hipMemcpy(dfi, fi.data(), 256 * sizeof(T), hipMemcpyHostToDevice));
    std::vector<Vt<T>> hy(nvec * 16);
    constexpr int TILES = 4;
    const int mblocks = nblocks;  // 16 * TILES = 64 vectors per wave, as one per lane in the butterfly
    for (int kind = 0; kind < 2; ++kind) {
        auto launch = [&](int reps) {
            if (kind == 0)
                hipLaunchKernelGGL((bfly_kernel<T>), dim3(nblocks), dim3(256), 0, 0, dx, dy, reps);
            else
                hipLaunchKernelGGL((mfma_kernel<T, TILES>), dim3(mblocks), dim3(256), 0, 0, dx, dy, dfr, dfi, reps);
            CK(hipGetLastError());
        };
        // one application against a direct DFT on the host (long double)
        launch(1);
        CK(hipDeviceSynchronize());
        CK(hipMemcpy(hy.data(), dy, nvec * 16 * sizeof(Vt<T>), hipMemcpyDeviceToHost));
        double maxerr = 0.0, maxref = 0.0;
        for (long v = 0; v < nvec; v += 997) {
            for (int k = 0; k < 15; ++k) {
                long double sr = 0, si = 0;
                for (int n = 0; n < 15; ++n) {
                    const long double a = 2.0L * 3.141592653589793238462643383279502884L * ((k * n) % 15) / 15.0L;
                    sr += hx[v * 16 + n].x * cosl(a) - hx[v * 16 + n].y * sinl(a);
                    si += hx[v * 16 + n].x * sinl(a) + hx[v * 16 + n].y * cosl(a);
                }
                maxerr = fmax(maxerr, fabs((double)(hy[v * 16 + k].x - sr)) + fabs((double)(hy[v * 16 + k].y - si)));
                maxref = fmax(maxref, fabs((double)sr) + fabs((double)si));
            }
        }
        hipEvent_t e0, e1;
        CK(hipEventCreate(&e0));
        CK(hipEventCreate(&e1));
        launch(reps_time);
        CK(hipEventRecord(e0, 0));
        const int runs = 10;
        for (int i = 0; i < runs; ++i) launch(reps_time);
        CK(hipEventRecord(e1, 0));
        CK(hipEventSynchronize(e1));
        float ms = 0;
        CK(hipEventElapsedTime(&ms, e0, e1));
        const double dfts = (double)nvec * reps_time * runs;
        printf("%s %s: rel err of one DFT %.2e; %d dependent DFT15 per vector, %ld vectors: %.3f ms per launch, %.2f G DFT15/s\n",
               name, kind == 0 ? "butterfly" : "mfma16x16x4", maxerr / maxref, reps_time, nvec, ms / runs,
               dfts / (ms * 1e-3) / 1e9);
        fflush(stdout);
    }
    CK(hipFree(dx));
    CK(hipFree(dy));
    CK(hipFree(dfr));
    CK(hipFree(dfi));
}

int main() {
    run<float>("fp32", 4096, 48);
    run<double>("fp64", 4096, 48);
    return 0;
}
