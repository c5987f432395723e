// Measurement probe, not part of the library: the vector-instruction issue
// rate of one MI355X for the instruction kinds the ray caster's loop is made
// of, as wave64 instructions per SIMD per clock.  The roofline of the caster
// (bound by vector issue, not by HBM) is taken against the peak these rates
// come close to.
//
// Each kernel runs long unrolled chains of one kind (8 independent chains per
// lane, inline asm so the count is exact), at 8 wavefronts per SIMD, and is
// timed with HIP events; the SIMD clock is read on the device (s_memtime
// against the 100 MHz s_memrealtime), since a full FMA load lowers it.
// Prints one JSON object.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

namespace {

constexpr int kIters = 2000;
constexpr int kUnroll = 8;

template <int KIND>
__global__ __launch_bounds__(256) void k_probe(uint32_t* out, uint64_t* clk) {
  uint32_t a0 = threadIdx.x, a1 = a0 + 1, a2 = a0 + 2, a3 = a0 + 3, a4 = a0 + 4, a5 = a0 + 5,
           a6 = a0 + 6, a7 = a0 + 7;
  uint32_t b = blockIdx.x | 1u;
  float f0 = (float)a0, f1 = f0 + 1, f2 = f0 + 2, f3 = f0 + 3, f4 = f0 + 4, f5 = f0 + 5,
        f6 = f0 + 6, f7 = f0 + 7;
  float fb = 1.0001f, fc = 0.5f;
  double d0 = a0, d1 = d0 + 1, d2 = d0 + 2, d3 = d0 + 3;
  const double db = 1.0001, dc = 0.5;
  const uint64_t t0 = __builtin_amdgcn_s_memtime(), r0 = __builtin_amdgcn_s_memrealtime();
  for (int i = 0; i < kIters; ++i) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      if constexpr (KIND == 0) {  // 8 x v_add_u32 (integer add)
        asm volatile(
            "v_add_u32 %0, %0, %8\n v_add_u32 %1, %1, %8\n v_add_u32 %2, %2, %8\n"
            "v_add_u32 %3, %3, %8\n v_add_u32 %4, %4, %8\n v_add_u32 %5, %5, %8\n"
            "v_add_u32 %6, %6, %8\n v_add_u32 %7, %7, %8"
            : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6), "+v"(a7)
            : "v"(b));
      } else if constexpr (KIND == 1) {  // 8 x v_fma_f32
        asm volatile(
            "v_fma_f32 %0, %0, %8, %9\n v_fma_f32 %1, %1, %8, %9\n v_fma_f32 %2, %2, %8, %9\n"
            "v_fma_f32 %3, %3, %8, %9\n v_fma_f32 %4, %4, %8, %9\n v_fma_f32 %5, %5, %8, %9\n"
            "v_fma_f32 %6, %6, %8, %9\n v_fma_f32 %7, %7, %8, %9"
            : "+v"(f0), "+v"(f1), "+v"(f2), "+v"(f3), "+v"(f4), "+v"(f5), "+v"(f6), "+v"(f7)
            : "v"(fb), "v"(fc));
      } else if constexpr (KIND == 2) {  // 8 x v_mov_b32
        asm volatile(
            "v_mov_b32 %0, %1\n v_mov_b32 %1, %2\n v_mov_b32 %2, %3\n v_mov_b32 %3, %4\n"
            "v_mov_b32 %4, %5\n v_mov_b32 %5, %6\n v_mov_b32 %6, %7\n v_mov_b32 %7, %0"
            : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6), "+v"(a7));
      } else if constexpr (KIND == 3) {  // the leaf step's mix: add, fma, select, convert,
                                         // mul, min, and, compare (one each)
        asm volatile(
            "v_add_u32 %0, %0, %5\n v_fma_f32 %6, %6, %9, %10\n v_cndmask_b32 %1, %1, %5, vcc\n"
            "v_cvt_f32_u32 %7, %2\n v_mul_f32 %8, %8, %9\n v_min_f32 %11, %11, %10\n"
            "v_and_b32 %3, %3, %5\n v_cmp_gt_u32 vcc, %4, %5"
            : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(b), "+v"(f0), "+v"(f1),
              "+v"(f2), "+v"(fb), "+v"(fc), "+v"(f3)
            :
            : "vcc");
      } else if constexpr (KIND == 4) {  // 4 x v_fma_f64
        asm volatile(
            "v_fma_f64 %0, %0, %4, %5\n v_fma_f64 %1, %1, %4, %5\n v_fma_f64 %2, %2, %4, %5\n"
            "v_fma_f64 %3, %3, %4, %5"
            : "+v"(d0), "+v"(d1), "+v"(d2), "+v"(d3)
            : "v"(db), "v"(dc));
      } else {  // 8 x v_exp_f32 (transcendental)
        asm volatile(
            "v_exp_f32 %0, %0\n v_exp_f32 %1, %1\n v_exp_f32 %2, %2\n v_exp_f32 %3, %3\n"
            "v_exp_f32 %4, %4\n v_exp_f32 %5, %5\n v_exp_f32 %6, %6\n v_exp_f32 %7, %7"
            : "+v"(f0), "+v"(f1), "+v"(f2), "+v"(f3), "+v"(f4), "+v"(f5), "+v"(f6), "+v"(f7));
      }
    }
  }
  const uint64_t t1 = __builtin_amdgcn_s_memtime(), r1 = __builtin_amdgcn_s_memrealtime();
  const uint32_t s = a0 ^ a1 ^ a2 ^ a3 ^ a4 ^ a5 ^ a6 ^ a7 ^
                     __float_as_uint(f0 + f1 + f2 + f3 + f4 + f5 + f6 + f7) ^
                     (uint32_t)__double_as_longlong(d0 + d1 + d2 + d3);
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    clk[0] = t1 - t0;
    clk[1] = r1 - r0;
  }
}

const char* const kNames[] = {"v_add_u32", "v_fma_f32", "v_mov_b32", "leaf_mix", "v_fma_f64",
                              "v_exp_f32"};
const int kPerUnroll[] = {8, 8, 8, 8, 4, 8};

int g_err = 0;

template <int KIND>
void run(int n_cu, uint32_t* out, uint64_t* clk, bool comma) {
  const int wg = 256, waves_per_cu = 32;  // 8 wavefronts per SIMD
  const int blocks = n_cu * waves_per_cu * 64 / wg;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    g_err = 1;
    return;
  }
  hipLaunchKernelGGL(k_probe<KIND>, dim3(blocks), dim3(wg), 0, 0, out, clk);
  float best = 1e30f;
  for (int r = 0; r < 3 && hipDeviceSynchronize() == hipSuccess; ++r) {
    (void)hipEventRecord(e0);
    hipLaunchKernelGGL(k_probe<KIND>, dim3(blocks), dim3(wg), 0, 0, out, clk);
    (void)hipEventRecord(e1);
    float ms = 0.0f;
    if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      g_err = 1;
      break;
    }
    best = ms < best ? ms : best;
  }
  uint64_t c[2] = {0, 1};
  if (hipMemcpy(c, clk, sizeof(c), hipMemcpyDeviceToHost) != hipSuccess) g_err = 1;
  const double instr = (double)blocks * wg / 64 * kIters * kUnroll * kPerUnroll[KIND];
  const double ghz = (double)c[0] / ((double)c[1] / 100e6) / 1e9;
  const double simd = 4.0 * n_cu;
  std::printf("%s\"%s\": {\"ms\": %.4f, \"per_simd_cycle_at_2.4GHz\": %.4f, "
              "\"measured_GHz\": %.3f, \"per_simd_cycle_at_measured_clock\": %.4f}",
              comma ? ", " : "", kNames[KIND], best, instr / (simd * 2.4e9 * best * 1e-3), ghz,
              instr / (simd * ghz * 1e9 * best * 1e-3));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}

}  // namespace

int main() {
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, 0) != hipSuccess) return 1;
  const int n_cu = p.multiProcessorCount;
  uint32_t* out = nullptr;
  uint64_t* clk = nullptr;
  if (hipMalloc(&out, (size_t)n_cu * 32 * 64 * sizeof(uint32_t)) != hipSuccess) return 1;
  if (hipMalloc(&clk, 2 * sizeof(uint64_t)) != hipSuccess) return 1;
  std::printf("{\"arch\": \"%s\", \"cu\": %d, \"waves_per_simd\": 8, ", p.gcnArchName, n_cu);
  run<0>(n_cu, out, clk, false);
  run<1>(n_cu, out, clk, true);
  run<2>(n_cu, out, clk, true);
  run<3>(n_cu, out, clk, true);
  run<4>(n_cu, out, clk, true);
  run<5>(n_cu, out, clk, true);
  std::printf("}\n");
  (void)hipFree(out);
  (void)hipFree(clk);
  return g_err;
}
