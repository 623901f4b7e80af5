// fio_calibrate: measurement aid for the roofline figures of the library.
//   fio_calibrate copy   1 GiB device-to-device copy kernel (known bytes), used to
//                        scale the FETCH_SIZE / WRITE_SIZE counters of rocprofv3;
//   fio_calibrate mfma   sustained 16x16x4 FP32 and FP64 MFMA rates (registers only;
//                        16 and 8 independent accumulators per wave: the FP64 loop
//                        is slower with 16, and below what the FP64 stage kernels
//                        reach, so it bounds the FP64 rate from below only);
//   fio_calibrate read   streaming read of 4 GiB (16-byte loads, eight in flight per
//                        lane, one partial sum written per workgroup): the HBM read
//                        rate a bandwidth-bound kernel can reach in practice.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) calib_copy(const float4 *__restrict__ a, float4 *__restrict__ b, long n) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) b[i] = a[i];
}

__global__ void __launch_bounds__(256) calib_read(const float4 *__restrict__ a, float *__restrict__ out, long n) {
    float4 s = {0.f, 0.f, 0.f, 0.f};
    const long stride = (long)gridDim.x * blockDim.x;
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    for (; i + 7 * stride < n; i += 8 * stride) {
        float4 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = a[i + u * stride];
#pragma unroll
        for (int u = 0; u < 8; ++u) { s.x += v[u].x; s.y += v[u].y; s.z += v[u].z; s.w += v[u].w; }
    }
    for (; i < n; i += stride) { const float4 v = a[i]; s.x += v.x; s.y += v.y; s.z += v.z; s.w += v.w; }
    __shared__ float red[256];
    red[threadIdx.x] = s.x + s.y + s.z + s.w;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.f;
        for (int k = 0; k < 256; ++k) t += red[k];
        out[blockIdx.x] = t;
    }
}

template <int NACC>
__global__ void __launch_bounds__(256) calib_mfma32(float *out, int iters, float a0) {
    floatx4 acc[NACC];
    for (int i = 0; i < NACC; ++i) acc[i] = floatx4{0, 0, 0, 0};
    float a = a0 + threadIdx.x * 1e-6f, b = a0 - threadIdx.x * 1e-6f;
    for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int i = 0; i < NACC; ++i) acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[i], 0, 0, 0);
    float s = 0;
    for (int i = 0; i < NACC; ++i) s += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
    if (s == 12345.f) out[threadIdx.x] = s;
}

template <int NACC>
__global__ void __launch_bounds__(256) calib_mfma64(double *out, int iters, double a0) {
    doublex4 acc[NACC];
    for (int i = 0; i < NACC; ++i) acc[i] = doublex4{0, 0, 0, 0};
    double a = a0 + threadIdx.x * 1e-6, b = a0 - threadIdx.x * 1e-6;
    for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int i = 0; i < NACC; ++i) acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[i], 0, 0, 0);
    double s = 0;
    for (int i = 0; i < NACC; ++i) s += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
    if (s == 12345.0) out[threadIdx.x] = s;
}

#define CK(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) { fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_)); return 1; } } while (0)

int main(int argc, char **argv) {
    const char *mode = argc > 1 ? argv[1] : "copy";
    hipEvent_t e0, e1;
    CK(hipEventCreate(&e0));
    CK(hipEventCreate(&e1));
    float ms = 0;
    if (!strcmp(mode, "copy")) {
        const long n = 1L << 26;  // float4 elements: 1 GiB per buffer
        float4 *a, *b;
        CK(hipMalloc(&a, n * 16));
        CK(hipMalloc(&b, n * 16));
        CK(hipMemset(a, 0, n * 16));
        hipLaunchKernelGGL(calib_copy, dim3(4096), dim3(256), 0, 0, a, b, n);
        CK(hipDeviceSynchronize());
        const int reps = 5;
        CK(hipEventRecord(e0));
        for (int r = 0; r < reps; ++r) hipLaunchKernelGGL(calib_copy, dim3(4096), dim3(256), 0, 0, a, b, n);
        CK(hipEventRecord(e1));
        CK(hipEventSynchronize(e1));
        CK(hipEventElapsedTime(&ms, e0, e1));
        printf("copy: 1 GiB read + 1 GiB write per dispatch, %.2f TB/s\n", 2.0 * n * 16 * reps / ms / 1e9);
        CK(hipFree(a));
        CK(hipFree(b));
    } else if (!strcmp(mode, "read")) {
        const long n = 1L << 28;  // float4 elements: 4 GiB
        float4 *a;
        float *o;
        CK(hipMalloc(&a, n * 16));
        CK(hipMalloc(&o, 65536 * sizeof(float)));
        CK(hipMemset(a, 0, n * 16));
        for (int blocks : {4096, 16384, 65536}) {
            hipLaunchKernelGGL(calib_read, dim3(blocks), dim3(256), 0, 0, a, o, n);
            CK(hipDeviceSynchronize());
            const int reps = 5;
            CK(hipEventRecord(e0));
            for (int r = 0; r < reps; ++r) hipLaunchKernelGGL(calib_read, dim3(blocks), dim3(256), 0, 0, a, o, n);
            CK(hipEventRecord(e1));
            CK(hipEventSynchronize(e1));
            CK(hipEventElapsedTime(&ms, e0, e1));
            printf("read: 4 GiB per dispatch, %d workgroups, %.2f TB/s\n", blocks, 1.0 * n * 16 * reps / ms / 1e9);
        }
        CK(hipFree(a));
        CK(hipFree(o));
    } else {
        float *o;
        double *od;
        CK(hipMalloc(&o, 4096));
        CK(hipMalloc(&od, 8192));
        const int iters = 2000, blocks = 2048;
        hipLaunchKernelGGL(calib_mfma32<16>, dim3(blocks), dim3(256), 0, 0, o, 10, 1.0f);
        CK(hipDeviceSynchronize());
        CK(hipEventRecord(e0));
        hipLaunchKernelGGL(calib_mfma32<16>, dim3(blocks), dim3(256), 0, 0, o, iters, 1.0f);
        CK(hipEventRecord(e1));
        CK(hipEventSynchronize(e1));
        CK(hipEventElapsedTime(&ms, e0, e1));
        printf("mfma f32 16x16x4: %.1f TFLOP/s\n", 2048.0 * 16 * iters * blocks * 4 / ms / 1e9);
        hipLaunchKernelGGL(calib_mfma64<8>, dim3(blocks), dim3(256), 0, 0, od, 10, 1.0);
        CK(hipDeviceSynchronize());
        CK(hipEventRecord(e0));
        hipLaunchKernelGGL(calib_mfma64<8>, dim3(blocks), dim3(256), 0, 0, od, iters, 1.0);
        CK(hipEventRecord(e1));
        CK(hipEventSynchronize(e1));
        CK(hipEventElapsedTime(&ms, e0, e1));
        printf("mfma f64 16x16x4: %.1f TFLOP/s\n", 2048.0 * 8 * iters * blocks * 4 / ms / 1e9);
    }
    return 0;
}
