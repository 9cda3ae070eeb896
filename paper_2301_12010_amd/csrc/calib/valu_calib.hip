// valu_calib.hip - calibration of the vector ALU ceiling that bounds the
// stage kernel (a measurement helper for the benchmark, not part of the
// solver's ABI; built into libswe_calib.so).
//
// Each thread runs 16 independent dependency chains for `iters` iterations.
// One iteration of one chain issues
//   op 0: two v_fma_f32                      (plain FP32 rate)
//   op 1: one v_rcp_f32 and one v_fma_f32    (transcendental rate)
//   op 2: one v_rcp_f32 and seven v_fma_f32  (about the stage kernel's mix)
// and nothing else executes in the loop, so the launch issues
// blocks x 4 waves x iters x 16 x (2 or 8) wave64 VALU instructions.
// The number of 256-thread blocks resident per CU, hence the waves per SIMD,
// is set by the static LDS of the instance (144, 72, 36 or 18 KB of the
// CU's 160 KB).  Packed FP32 is disabled for all device code, as for the
// solver, so the figure is the ceiling for the code this library runs.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

template <int OP, int LDSF>
__global__ __launch_bounds__(256) void k_valu(float *out, int iters, float a, float b)
{
    __shared__ float pad[LDSF];
    float x[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) x[k] = 1.0f + 0.01f * (float)(threadIdx.x + k);
    // touch the LDS so that its allocation, which sets the occupancy, stays
    pad[threadIdx.x] = x[0];
    __syncthreads();
    x[0] += pad[(threadIdx.x + 1) & 255] * 1e-9f;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            if (OP == 0) {
                x[k] = fmaf(x[k], a, b);
                x[k] = fmaf(x[k], a, b);
            } else {
                x[k] = __builtin_amdgcn_rcpf(x[k]);
#pragma unroll
                for (int j = 0; j < (OP == 1 ? 1 : 7); ++j) x[k] = fmaf(x[k], a, b);
            }
        }
    }
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < 16; ++k) s += x[k];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}

template <int OP>
hipError_t launch(int waves_per_simd, int blocks, int iters, float *out, hipStream_t st)
{
    const float a = 0.999f, b = 0.001f;
    switch (waves_per_simd) {
    case 1: hipLaunchKernelGGL((k_valu<OP, 36000>), dim3(blocks), dim3(256), 0, st, out, iters, a, b); break;
    case 2: hipLaunchKernelGGL((k_valu<OP, 18000>), dim3(blocks), dim3(256), 0, st, out, iters, a, b); break;
    case 4: hipLaunchKernelGGL((k_valu<OP, 9000>), dim3(blocks), dim3(256), 0, st, out, iters, a, b); break;
    default: hipLaunchKernelGGL((k_valu<OP, 4500>), dim3(blocks), dim3(256), 0, st, out, iters, a, b); break;
    }
    return hipGetLastError();
}

}  // namespace

extern "C" {

// Times one launch of the calibration kernel (after one untimed launch) on
// the current device and reports its duration and the wave64 VALU
// instructions its loops issue.  op: 0, 1 or 2 as above; waves_per_simd: 1,
// 2, 4 or 8; iters >= 1.  The grid holds 4 rounds of resident blocks on every
// CU.  Returns 0, -1 for invalid arguments, or the HIP error code.  Allocates
// and frees its own output buffer (blocks x 256 floats).
int swe_calib_valu(int32_t op, int32_t waves_per_simd, int32_t iters, float *ms, double *wave_instr)
{
    if (op < 0 || op > 2 || iters < 1 || !ms || !wave_instr) return -1;
    if (waves_per_simd != 1 && waves_per_simd != 2 && waves_per_simd != 4 && waves_per_simd != 8) return -1;
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return (int)e;
    const int blocks = cus * waves_per_simd * 4;
    float *out = nullptr;
    if ((e = hipMalloc(&out, (size_t)blocks * 256 * sizeof(float))) != hipSuccess) return (int)e;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto run = [&]() {
        return op == 0 ? launch<0>(waves_per_simd, blocks, iters, out, st)
                       : op == 1 ? launch<1>(waves_per_simd, blocks, iters, out, st)
                                 : launch<2>(waves_per_simd, blocks, iters, out, st);
    };
    if ((e = hipStreamCreate(&st)) == hipSuccess && (e = hipEventCreate(&e0)) == hipSuccess &&
        (e = hipEventCreate(&e1)) == hipSuccess && (e = run()) == hipSuccess &&
        (e = hipEventRecord(e0, st)) == hipSuccess && (e = run()) == hipSuccess &&
        (e = hipEventRecord(e1, st)) == hipSuccess && (e = hipEventSynchronize(e1)) == hipSuccess) {
        e = hipEventElapsedTime(ms, e0, e1);
        const double per_iter = op == 0 ? 2.0 : op == 1 ? 2.0 : 8.0;
        *wave_instr = (double)blocks * 4.0 * (double)iters * 16.0 * per_iter;
    }
    if (e1) (void)hipEventDestroy(e1);
    if (e0) (void)hipEventDestroy(e0);
    if (st) (void)hipStreamDestroy(st);
    (void)hipFree(out);
    return (int)e;
}

}  // extern "C"
