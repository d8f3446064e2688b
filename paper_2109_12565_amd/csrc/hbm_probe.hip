// Streaming HBM bandwidth probe for one GPU: copy, read-only and write-only
// passes over 1 GiB buffers with 16-byte accesses, plus a copy with 4-byte
// accesses (the width the lattice kernel uses). It gives the practical
// ceiling that the lattice kernel's HBM traffic is compared against; the
// nominal peak of the part is 8 TB/s.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

typedef float v4f __attribute__((ext_vector_type(4)));

#define CHECK(x)                                                              \
  do {                                                                        \
    hipError_t e_ = (x);                                                      \
    if (e_ != hipSuccess) {                                                   \
      std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));            \
      std::exit(1);                                                           \
    }                                                                         \
  } while (0)

__global__ void copy_plain(const v4f* __restrict__ a, v4f* __restrict__ b, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}
__global__ void copy_nt(const v4f* __restrict__ a, v4f* __restrict__ b, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    __builtin_nontemporal_store(__builtin_nontemporal_load(a + i), b + i);
}
__global__ void read_only(const v4f* __restrict__ a, float* __restrict__ sink, size_t n) {
  float s = 0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const v4f v = a[i];
    s += v.x + v.y + v.z + v.w;
  }
  if (s == 123.5f) sink[0] = s;  // never true for the zero-filled input
}
__global__ void write_nt(v4f* __restrict__ b, size_t n) {
  const v4f v = {1.f, 2.f, 3.f, 4.f};
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    __builtin_nontemporal_store(v, b + i);
}
__global__ void copy_f32_nt(const float* __restrict__ a, float* __restrict__ b, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    __builtin_nontemporal_store(a[i], b + i);
}

int main() {
  const size_t bytes = (size_t)1 << 30;
  const size_t n4 = bytes / sizeof(v4f), n1 = bytes / sizeof(float);
  v4f *a = nullptr, *b = nullptr;
  float* sink = nullptr;
  CHECK(hipMalloc(&a, bytes));
  CHECK(hipMalloc(&b, bytes));
  CHECK(hipMalloc(&sink, 64));
  CHECK(hipMemset(a, 0, bytes));
  CHECK(hipMemset(b, 0, bytes));
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  const char* names[] = {"copy", "copy_nt", "read", "write_nt", "copy_f32_nt"};
  std::printf("{\"probe\": \"hbm\", \"bytes_per_buffer\": %zu, \"results\": [", bytes);
  bool first = true;
  for (int grid : {1024, 2048, 4096, 16384}) {
    for (int kind = 0; kind < 5; ++kind) {
      auto launch = [&]() {
        switch (kind) {
          case 0: hipLaunchKernelGGL(copy_plain, dim3(grid), dim3(256), 0, 0, a, b, n4); break;
          case 1: hipLaunchKernelGGL(copy_nt, dim3(grid), dim3(256), 0, 0, a, b, n4); break;
          case 2: hipLaunchKernelGGL(read_only, dim3(grid), dim3(256), 0, 0, a, sink, n4); break;
          case 3: hipLaunchKernelGGL(write_nt, dim3(grid), dim3(256), 0, 0, b, n4); break;
          default:
            hipLaunchKernelGGL(copy_f32_nt, dim3(grid), dim3(256), 0, 0, (const float*)a, (float*)b, n1);
        }
      };
      launch();
      CHECK(hipGetLastError());
      CHECK(hipDeviceSynchronize());
      CHECK(hipEventRecord(e0));
      for (int it = 0; it < 10; ++it) launch();
      CHECK(hipEventRecord(e1));
      CHECK(hipEventSynchronize(e1));
      float ms = 0;
      CHECK(hipEventElapsedTime(&ms, e0, e1));
      ms /= 10;
      const double moved = (kind == 2 || kind == 3) ? (double)bytes : 2.0 * bytes;
      std::printf("%s{\"kernel\": \"%s\", \"grid\": %d, \"us\": %.1f, \"GBps\": %.1f}", first ? "" : ", ",
                  names[kind], grid, ms * 1e3, moved / ms / 1e6);
      first = false;
    }
  }
  std::printf("]}\n");
  return 0;
}
