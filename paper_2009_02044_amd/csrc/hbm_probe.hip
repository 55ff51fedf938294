// Memory-bandwidth probe for one GPU: streams of 16-byte loads and stores over 2 GiB buffers
// (read only, write only, copy; ordinary and non-temporal), grid-stride loops over 8
// work-groups of 256 threads per CU, timed with HIP events, best of 10.  It gives the achievable ceilings against which the step
// kernels' HBM fractions are read (the nominal peak is 8 TB/s).
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdlib>

namespace {

constexpr int BS = 256;
using v4 = unsigned __attribute__((ext_vector_type(4)));   // 16 bytes

// NT: non-temporal loads and stores (as the step kernels' own-site data and outputs)
template <bool NT> __device__ __forceinline__ v4 ld(const v4* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <bool NT> __device__ __forceinline__ void st(v4 v, v4* p) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// Each thread makes U 16-byte accesses per loop trip (i, i + stride, ..., all guarded), a
// grid-stride loop over the buffer.  U = 1 measures fastest: with U = 4 the non-temporal read
// drops from 7.2 to 6.1 TB/s.
constexpr int U = 1;

template <bool NT>
__global__ void __launch_bounds__(BS) k_read(const v4* __restrict__ src, size_t n, unsigned* __restrict__ out) {
  unsigned acc = 0;
  const size_t stride = (size_t)gridDim.x * BS;
  for (size_t i = (size_t)blockIdx.x * BS + threadIdx.x; i < n; i += U * stride) {
    v4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (i + u * stride < n) v[u] = ld<NT>(&src[i + u * stride]);
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (i + u * stride < n) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
  }
  out[(size_t)blockIdx.x * BS + threadIdx.x] = acc;   // keeps the loads
}

template <bool NT> __global__ void __launch_bounds__(BS) k_write(v4* __restrict__ dst, size_t n) {
  const size_t stride = (size_t)gridDim.x * BS;
  for (size_t i = (size_t)blockIdx.x * BS + threadIdx.x; i < n; i += U * stride) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t j = i + u * stride;
      if (j < n) {
        const unsigned k = (unsigned)j;
        const v4 v = {k, k + 1u, k + 2u, k + 3u};
        st<NT>(v, &dst[j]);
      }
    }
  }
}

// LNT / SNT: non-temporal loads / stores
template <bool LNT, bool SNT>
__global__ void __launch_bounds__(BS) k_copy(const v4* __restrict__ src, v4* __restrict__ dst, size_t n) {
  const size_t stride = (size_t)gridDim.x * BS;
  for (size_t i = (size_t)blockIdx.x * BS + threadIdx.x; i < n; i += U * stride) {
    v4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (i + u * stride < n) v[u] = ld<LNT>(&src[i + u * stride]);
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (i + u * stride < n) st<SNT>(v[u], &dst[i + u * stride]);
  }
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

int main() {
  const size_t bytes = (size_t)2 << 30;
  const size_t n = bytes / sizeof(v4);
  int dev = 0, cus = 0;
  CK(hipGetDevice(&dev));
  CK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int blocks = 8 * cus;
  v4 *a, *b;
  unsigned* sink;
  CK(hipMalloc(&a, bytes));
  CK(hipMalloc(&b, bytes));
  CK(hipMalloc(&sink, (size_t)blocks * BS * sizeof(unsigned)));
  CK(hipMemset(a, 1, bytes));
  CK(hipMemset(b, 2, bytes));
  hipEvent_t e0, e1;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  constexpr int NK = 8;
  const char* names[NK] = {"read ",
                           "write",
                           "copy ",
                           "read  (non-temporal)",
                           "write (non-temporal)",
                           "copy  (non-temporal)",
                           "copy  (nt loads)",
                           "copy  (nt stores)"};
  float best[NK];
  for (int k = 0; k < NK; ++k) best[k] = 1e30f;
  for (int rep = 0; rep < 10; ++rep) {
    for (int k = 0; k < NK; ++k) {
      CK(hipEventRecord(e0));
      switch (k) {
        case 0: k_read<false><<<blocks, BS>>>(a, n, sink); break;
        case 1: k_write<false><<<blocks, BS>>>(b, n); break;
        case 2: k_copy<false, false><<<blocks, BS>>>(a, b, n); break;
        case 3: k_read<true><<<blocks, BS>>>(a, n, sink); break;
        case 4: k_write<true><<<blocks, BS>>>(b, n); break;
        case 5: k_copy<true, true><<<blocks, BS>>>(a, b, n); break;
        case 6: k_copy<true, false><<<blocks, BS>>>(a, b, n); break;
        default: k_copy<false, true><<<blocks, BS>>>(a, b, n); break;
      }
      CK(hipGetLastError());
      CK(hipEventRecord(e1));
      CK(hipEventSynchronize(e1));
      float ms;
      CK(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best[k]) best[k] = ms;
    }
  }
  const double gb = (double)bytes / 1e9;
  std::printf("CUs %d, work-groups %d, buffer %.2f GB\n", cus, blocks, gb);
  for (int k = 0; k < NK; ++k) {
    const bool copy = k == 2 || k >= 5;
    const double moved = (copy ? 2 : 1) * gb;
    std::printf("%-22s %8.3f ms  %7.0f GB/s%s\n", names[k], best[k], moved / (best[k] * 1e-3),
                copy ? " (read + write bytes)" : "");
  }
  CK(hipFree(a));
  CK(hipFree(b));
  CK(hipFree(sink));
  return 0;
}
