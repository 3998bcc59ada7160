// Calibration of the FLOP accounting: a kernel of known fused multiply-add
// count, to measure what the vector ALUs sustain for the instruction forms the
// solver kernels are built from (single FP32 and FP64 FMAs; packed FP32 is
// disabled in every unit of this library) and to check what the hardware
// counters report for a known number of instructions and flops.
//
// Every lane runs C independent chains a <- a * b + c for `rounds` rounds of
// kRound steps each, so a launch issues exactly
//   (threads / 64) * rounds * kRound * C
// wave64 FMA instructions and twice as many flops per lane.  C = 1 exposes
// the FMA latency; larger C gives each wave independent work to issue back to
// back.  The number of resident waves per SIMD is set by the grid: one block of
// four waves per CU and per requested wave.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "../../include/hjpd.h"

int hjpd_fail(int code, const char* msg);

namespace {

constexpr int kRound = 32;

template <typename T, int C>
__global__ void __launch_bounds__(256) k_calib_fma(int64_t rounds, T b, T c, T* out) {
  T acc[C];
#pragma unroll
  for (int i = 0; i < C; i++) acc[i] = T(threadIdx.x & 7) + T(i);
  for (int64_t r = 0; r < rounds; r++) {
#pragma unroll
    for (int u = 0; u < kRound; u++)
#pragma unroll
      for (int i = 0; i < C; i++) acc[i] = std::fma(acc[i], b, c);
  }
  T s = T(0);
#pragma unroll
  for (int i = 0; i < C; i++) s += acc[i];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

template <typename T>
const void* calib_kernel(int chains) {
  switch (chains) {
    case 1: return reinterpret_cast<const void*>(&k_calib_fma<T, 1>);
    case 2: return reinterpret_cast<const void*>(&k_calib_fma<T, 2>);
    case 4: return reinterpret_cast<const void*>(&k_calib_fma<T, 4>);
    case 8: return reinterpret_cast<const void*>(&k_calib_fma<T, 8>);
    case 16: return reinterpret_cast<const void*>(&k_calib_fma<T, 16>);
    default: return nullptr;
  }
}

}  // namespace

#define CAL_OK(expr, what)                                                          \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess) {                                                         \
      rc = hjpd_fail(HJPD_EDEVICE, (std::string(what) + ": " + hipGetErrorString(e_)).c_str()); \
      goto done;                                                                    \
    }                                                                               \
  } while (0)

extern "C" int hjpd_calibrate_fma(int dtype, int chains, int waves_per_simd, int64_t rounds, double* ms,
                                  double* flops, double* wave_instructions) {
  if (!ms || (dtype != HJPD_F32 && dtype != HJPD_F64) || rounds < 1 || rounds > (int64_t(1) << 30) ||
      waves_per_simd < 1 || waves_per_simd > 8)
    return hjpd_fail(HJPD_EINVAL, "calibrate_fma: bad argument");
  const void* k = dtype == HJPD_F32 ? calib_kernel<float>(chains) : calib_kernel<double>(chains);
  if (!k) return hjpd_fail(HJPD_EINVAL, "calibrate_fma: chains must be 1, 2, 4, 8 or 16");
  int rc = HJPD_OK;
  int dev = 0, cus = 0;
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  void* out = nullptr;
  float t = 0.f;
  const size_t esz = dtype == HJPD_F32 ? sizeof(float) : sizeof(double);
  {
    CAL_OK(hipGetDevice(&dev), "hipGetDevice");
    CAL_OK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "CU count");
    const unsigned blocks = unsigned(cus) * unsigned(waves_per_simd);
    CAL_OK(hipMalloc(&out, size_t(blocks) * 256 * esz), "hipMalloc");
    CAL_OK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "hipStreamCreate");
    CAL_OK(hipEventCreate(&e0), "hipEventCreate");
    CAL_OK(hipEventCreate(&e1), "hipEventCreate");
    // b < 1 keeps every chain bounded (it tends to c / (1 - b))
    const double b = 0.999999, c = 1e-6;
    for (int rep = 0; rep < 2; rep++) {  // the first launch warms up, the second is timed
      if (rep == 1) CAL_OK(hipEventRecord(e0, s), "hipEventRecord");
      if (dtype == HJPD_F32) {
        float bf = float(b), cf = float(c);
        float* o = static_cast<float*>(out);
        void* args[] = {&rounds, &bf, &cf, &o};
        CAL_OK(hipLaunchKernel(k, dim3(blocks), dim3(256), args, 0, s), "launch");
      } else {
        double bd = b, cd = c;
        double* o = static_cast<double*>(out);
        void* args[] = {&rounds, &bd, &cd, &o};
        CAL_OK(hipLaunchKernel(k, dim3(blocks), dim3(256), args, 0, s), "launch");
      }
      if (rep == 1) CAL_OK(hipEventRecord(e1, s), "hipEventRecord");
    }
    CAL_OK(hipEventSynchronize(e1), "hipEventSynchronize");
    CAL_OK(hipEventElapsedTime(&t, e0, e1), "hipEventElapsedTime");
    const double insts = double(blocks) * 4.0 * double(rounds) * kRound * chains;
    *ms = t;
    if (flops) *flops = insts * 64.0 * 2.0;
    if (wave_instructions) *wave_instructions = insts;
  }
done:
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (s) (void)hipStreamDestroy(s);
  if (out) (void)hipFree(out);
  return rc;
}
