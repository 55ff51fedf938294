// Issue-rate probe for gfx950 vector instructions: how many cycles one wave64 instruction holds
// its SIMD, per instruction form.  Each kernel runs 8 independent dependency chains per lane
// (no latency stalls at 16 waves per CU) of one instruction form, the same count in every
// kernel: 8 n instructions per wavefront.  Timed with HIP events here; cycles per instruction
// come from the counters (GRBM_GUI_ACTIVE / 8 XCDs over SQ_INSTS_VALU / 1024 SIMDs) when it
// runs under rocprofv3 --pmc.  It backs the issue model used for the step kernels' VALU-busy
// figures (FP64 and 32-bit integer: 4 cycles; FP32 with vector operands: about 2).
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdlib>

namespace {

constexpr int BS = 256;

template <typename T> __device__ __forceinline__ T fma_(T a, T b, T c);
template <> __device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <> __device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T> __device__ __forceinline__ void store_sum(T* out, const T (&a)[8]) {
  T s = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) s += a[i];
  out[blockIdx.x * BS + threadIdx.x] = s;
}

// a <- a b + c with b, c uniform: VOP3 fma reading a scalar register every time
template <typename T> __global__ void __launch_bounds__(BS) k_fma_sgpr(T* out, T b, T c, int n) {
  T a[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) a[i] = (T)(threadIdx.x + i);
  for (int it = 0; it < n; ++it) {
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] = fma_(a[i], b, c);
  }
  store_sum(out, a);
}

// a <- x y + a, all vector registers: the two-operand accumulate form (v_fmac)
template <typename T> __global__ void __launch_bounds__(BS) k_fmac(T* out, T b, int n) {
  T a[8], x[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    a[i] = (T)(threadIdx.x + i);
    x[i] = (T)(threadIdx.x * 3 + i) * b;
  }
  for (int it = 0; it < n; ++it) {
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] = fma_(x[i], x[(i + 1) & 7], a[i]);
  }
  store_sum(out, a);
}

// a <- a x + c, all vector registers, the addend kept: the three-operand form (VOP3 v_fma)
__global__ void __launch_bounds__(BS) k_fma3(float* out, float b, int n) {
  float a[8], x[8], c[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    a[i] = (float)(threadIdx.x + i);
    x[i] = (float)(1.0 + 1e-7 * i) * b;
    c[i] = 1e-3f * (float)(threadIdx.x * 5 + i);
  }
  for (int it = 0; it < n; ++it) {
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] = __builtin_fmaf(a[i], x[i], c[i]);
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) a[i] += c[i] + x[i];
  store_sum(out, a);
}

// a <- -x y + a: a negation modifier on a vector operand (VOP3 form)
__global__ void __launch_bounds__(BS) k_fma_neg(float* out, float b, int n) {
  float a[8], x[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    a[i] = (float)(threadIdx.x + i);
    x[i] = (float)(threadIdx.x * 3 + i) * b;
  }
  for (int it = 0; it < n; ++it) {
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] = __builtin_fmaf(-x[i], x[(i + 1) & 7], a[i]);
  }
  store_sum(out, a);
}

// a <- a x, vector registers (one chain of eight also reads the scalar b)
__global__ void __launch_bounds__(BS) k_mul(float* out, float b, int n) {
  float a[8], x[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    a[i] = (float)(threadIdx.x + i);
    x[i] = (float)(1.0 + 1e-7 * i) * b;
  }
  for (int it = 0; it < n; ++it) {
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] = a[i] * x[i];
  }
  store_sum(out, a);
}

// 32-bit integer: a <- (a ^ b) + i (one v_xad_u32 each)
__global__ void __launch_bounds__(BS) k_u32(unsigned* out, unsigned b, int n) {
  unsigned a[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) a[i] = threadIdx.x * 7u + (unsigned)i;
  for (int it = 0; it < n; ++it) {
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] = (a[i] ^ b) + (unsigned)i;
  }
  store_sum(out, a);
}

#define CK(x)                                                                                   \
  do {                                                                                          \
    hipError_t e_ = (x);                                                                        \
    if (e_ != hipSuccess) {                                                                     \
      std::printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__);              \
      std::exit(1);                                                                             \
    }                                                                                           \
  } while (0)

}  // namespace

int main(int argc, char** argv) {
  const int blocks = 4096;   // 16 waves per CU on 256 CUs
  const int n = argc > 1 ? std::atoi(argv[1]) : 20000;
  if (n <= 0) {
    std::printf("usage: valu_probe [iterations > 0]\n");
    return 2;
  }
  void* buf;
  CK(hipMalloc(&buf, (size_t)blocks * BS * sizeof(double)));
  hipEvent_t e0, e1;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  const char* names[] = {"f64 fma (sgpr operand)", "f32 fma (sgpr operand)", "u32 xor+add",
                         "f32 fmac (vector)",      "f64 fmac (vector)",      "f32 mul (vector)",
                         "f32 fma (vector, vop3)", "f32 fma (negated operand)"};
  const double inst_per_simd = (double)blocks * (BS / 64) * 8 * n / 1024.0;
  for (int rep = 0; rep < 2; ++rep) {
    for (int k = 0; k < 8; ++k) {
      CK(hipEventRecord(e0));
      switch (k) {
        case 0: k_fma_sgpr<double><<<blocks, BS>>>((double*)buf, 0.999, 1e-3, n); break;
        case 1: k_fma_sgpr<float><<<blocks, BS>>>((float*)buf, 0.999f, 1e-3f, n); break;
        case 2: k_u32<<<blocks, BS>>>((unsigned*)buf, 0x9e3779b9u, n); break;
        case 3: k_fmac<float><<<blocks, BS>>>((float*)buf, 1e-3f, n); break;
        case 4: k_fmac<double><<<blocks, BS>>>((double*)buf, 1e-3, n); break;
        case 5: k_mul<<<blocks, BS>>>((float*)buf, 0.999999f, n); break;
        case 6: k_fma3<<<blocks, BS>>>((float*)buf, 0.999f, n); break;
        default: k_fma_neg<<<blocks, BS>>>((float*)buf, 1e-3f, n); break;
      }
      CK(hipGetLastError());
      CK(hipEventRecord(e1));
      CK(hipEventSynchronize(e1));
      float ms;
      CK(hipEventElapsedTime(&ms, e0, e1));
      std::printf("rep %d  %-26s %9.3f ms  %.4f wave-instructions per SIMD per ns\n", rep, names[k], ms,
                  inst_per_simd / (ms * 1e6));
    }
  }
  CK(hipFree(buf));
  return 0;
}
