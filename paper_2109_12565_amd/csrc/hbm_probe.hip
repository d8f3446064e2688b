// Streaming HBM bandwidth probe for one GPU: copy, read-only and write-only
// passes over 1 GiB buffers with 16-byte accesses, plus a copy with 4-byte
// accesses (the width the lattice kernel uses). It gives the practical
// ceiling that the lattice kernel's HBM traffic is compared against; the
// nominal peak of the part is 8 TB/s.
//
// Second part: the lattice step's memory pattern with its arithmetic taken
// out, on a 4096 x 2048 lattice of 27 FP32 planes: every node loads the 27
// values a pull step loads (x and y shifted by the direction's velocity,
// periodic in x, clamped at the walls) and stores 27 values
// (non-temporal), in 256-wide strips of 32 rows. Variants: plain block
// order; the step kernel's XCD-aware tile order with alternating chunk
// direction and one barrier per row; and an interleaved layout in which the
// 27 planes of each 64-column group of a row are contiguous.
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

constexpr int kPLx = 4096, kPLy = 2048, kPRows = 32, kPPlanes = 27;
__constant__ int kPcx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__constant__ int kPcy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

// Layout 0: planes [27][ly][lx]; layout 1: [ly][lx/64][27][64].
template <int kLayout>
__device__ inline size_t pattern_index(int row, int col, int p) {
  if (kLayout == 0) return ((size_t)p * kPLy + row) * kPLx + col;
  return ((size_t)row * (kPLx / 64) + (col >> 6)) * (kPPlanes * 64) + (size_t)p * 64 + (col & 63);
}

template <int kLayout, bool kOrder>
__global__ __launch_bounds__(256) void step_pattern(const float* __restrict__ src,
                                                    float* __restrict__ dst) {
  const int nbx = gridDim.x, ntiles = gridDim.x * gridDim.y;
  const int lin = blockIdx.y * nbx + blockIdx.x;
  int tile = lin;
  if (kOrder) {
    const int xcd = lin % 8;
    tile = xcd * (ntiles / 8) + min(xcd, ntiles % 8) + lin / 8;
  }
  const int chunk = tile / nbx, strip = tile - chunk * nbx;
  const int x = strip * 256 + threadIdx.x;  // grid covers x in [0, kPLx) exactly
  const int xm = x == 0 ? kPLx - 1 : x - 1, xp = x == kPLx - 1 ? 0 : x + 1;
  const bool down = kOrder && (chunk & 1);
  for (int k = 0; k < kPRows; ++k) {
    const int r = down ? chunk * kPRows + kPRows - 1 - k : chunk * kPRows + k;
    float acc = 0.f;
#pragma unroll
    for (int p = 0; p < kPPlanes; ++p) {
      const int i = p % 9;
      int sr = r - kPcy[i];
      sr = sr < 0 ? 0 : (sr >= kPLy ? kPLy - 1 : sr);
      const int sx = kPcx[i] > 0 ? xm : (kPcx[i] < 0 ? xp : x);
      acc += src[pattern_index<kLayout>(sr, sx, p)];
    }
    if (kOrder) __syncthreads();
#pragma unroll
    for (int p = 0; p < kPPlanes; ++p)
      __builtin_nontemporal_store(acc + (float)p, dst + pattern_index<kLayout>(r, x, p));
  }
}

// The same pull pattern on 2-byte values (16-bit storages), plane layout and
// step order: one column per lane with 2-byte loads and stores, or two
// columns per lane with 4-byte ones, where the pulls from x - 1 and x + 1
// take the neighbour column from the adjacent lane and the wavefront's edge
// lanes load the word beyond it.
__global__ __launch_bounds__(256) void step_pattern_h(const uint16_t* __restrict__ src,
                                                      uint16_t* __restrict__ dst) {
  const int nbx = gridDim.x, ntiles = gridDim.x * gridDim.y;
  const int lin = blockIdx.y * nbx + blockIdx.x;
  const int xcd = lin % 8;
  const int tile = xcd * (ntiles / 8) + min(xcd, ntiles % 8) + lin / 8;
  const int chunk = tile / nbx, strip = tile - chunk * nbx;
  const int x = strip * 256 + threadIdx.x;
  const int xm = x == 0 ? kPLx - 1 : x - 1, xp = x == kPLx - 1 ? 0 : x + 1;
  const bool down = chunk & 1;
  for (int k = 0; k < kPRows; ++k) {
    const int r = down ? chunk * kPRows + kPRows - 1 - k : chunk * kPRows + k;
    uint32_t acc = 0;
#pragma unroll
    for (int p = 0; p < kPPlanes; ++p) {
      const int i = p % 9;
      int sr = r - kPcy[i];
      sr = sr < 0 ? 0 : (sr >= kPLy ? kPLy - 1 : sr);
      const int sx = kPcx[i] > 0 ? xm : (kPcx[i] < 0 ? xp : x);
      acc += src[pattern_index<0>(sr, sx, p)];
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < kPPlanes; ++p)
      __builtin_nontemporal_store((uint16_t)(acc + p), dst + pattern_index<0>(r, x, p));
  }
}

__global__ __launch_bounds__(256) void step_pattern_h2(const uint32_t* __restrict__ src,
                                                       uint32_t* __restrict__ dst) {
  constexpr int kW = kPLx / 2;  // words per row
  const int nbx = gridDim.x, ntiles = gridDim.x * gridDim.y;
  const int lin = blockIdx.y * nbx + blockIdx.x;
  const int xcd = lin % 8;
  const int tile = xcd * (ntiles / 8) + min(xcd, ntiles % 8) + lin / 8;
  const int chunk = tile / nbx, strip = tile - chunk * nbx;
  const int w = strip * 256 + threadIdx.x;  // grid covers the words of a row exactly
  const int lane = threadIdx.x & 63;
  const int wm = w == 0 ? kW - 1 : w - 1, wp = w == kW - 1 ? 0 : w + 1;
  const bool down = chunk & 1;
  auto word = [&](int p, int row, int ww) { return ((size_t)p * kPLy + row) * kW + ww; };
  for (int k = 0; k < kPRows; ++k) {
    const int r = down ? chunk * kPRows + kPRows - 1 - k : chunk * kPRows + k;
    uint32_t a0 = 0, a1 = 0;  // columns 2w and 2w + 1
#pragma unroll
    for (int p = 0; p < kPPlanes; ++p) {
      const int i = p % 9;
      int sr = r - kPcy[i];
      sr = sr < 0 ? 0 : (sr >= kPLy ? kPLy - 1 : sr);
      const uint32_t own = src[word(p, sr, w)];
      if (kPcx[i] == 0) {
        a0 += own & 0xffffu;
        a1 += own >> 16;
      } else if (kPcx[i] > 0) {  // from x - 1: the left word's high half
        uint32_t left = __shfl_up(own, 1, 64);
        if (lane == 0) left = src[word(p, sr, wm)];
        a0 += left >> 16;
        a1 += own & 0xffffu;
      } else {  // from x + 1: the right word's low half
        uint32_t right = __shfl_down(own, 1, 64);
        if (lane == 63) right = src[word(p, sr, wp)];
        a0 += own >> 16;
        a1 += right & 0xffffu;
      }
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < kPPlanes; ++p)
      __builtin_nontemporal_store(((a0 + p) & 0xffffu) | ((a1 + p) << 16), dst + word(p, r, w));
  }
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
  std::printf("], \"step_pattern\": [");
  CHECK(hipFree(a));
  CHECK(hipFree(b));
  const size_t pbytes = (size_t)kPPlanes * kPLx * kPLy * sizeof(float);
  float *pa = nullptr, *pb = nullptr;
  CHECK(hipMalloc(&pa, pbytes));
  CHECK(hipMalloc(&pb, pbytes));
  CHECK(hipMemset(pa, 0, pbytes));
  CHECK(hipMemset(pb, 0, pbytes));
  const char* pnames[] = {"planes_plain_order", "planes_step_order", "interleaved_step_order"};
  const dim3 pgrid(kPLx / 256, kPLy / kPRows);
  for (int kind = 0; kind < 3; ++kind) {
    auto launch = [&]() {
      if (kind == 0) hipLaunchKernelGGL((step_pattern<0, false>), pgrid, dim3(256), 0, 0, pa, pb);
      else if (kind == 1) hipLaunchKernelGGL((step_pattern<0, true>), pgrid, dim3(256), 0, 0, pa, pb);
      else hipLaunchKernelGGL((step_pattern<1, true>), pgrid, dim3(256), 0, 0, pa, pb);
    };
    launch();
    CHECK(hipGetLastError());
    CHECK(hipDeviceSynchronize());
    CHECK(hipEventRecord(e0));
    for (int it = 0; it < 20; ++it) launch();
    CHECK(hipEventRecord(e1));
    CHECK(hipEventSynchronize(e1));
    float ms = 0;
    CHECK(hipEventElapsedTime(&ms, e0, e1));
    ms /= 20;
    std::printf("%s{\"kernel\": \"%s\", \"us\": %.1f, \"GBps\": %.1f}", kind ? ", " : "",
                pnames[kind], ms * 1e3, 2.0 * pbytes / ms / 1e6);
  }
  // 16-bit values: the same lattice, half the bytes
  const dim3 hgrid(kPLx / 256, kPLy / kPRows), h2grid(kPLx / 512, kPLy / kPRows);
  for (int kind = 0; kind < 2; ++kind) {
    auto launch = [&]() {
      if (kind == 0)
        hipLaunchKernelGGL(step_pattern_h, hgrid, dim3(256), 0, 0, (const uint16_t*)pa, (uint16_t*)pb);
      else
        hipLaunchKernelGGL(step_pattern_h2, h2grid, dim3(256), 0, 0, (const uint32_t*)pa, (uint32_t*)pb);
    };
    launch();
    CHECK(hipGetLastError());
    CHECK(hipDeviceSynchronize());
    CHECK(hipEventRecord(e0));
    for (int it = 0; it < 20; ++it) launch();
    CHECK(hipEventRecord(e1));
    CHECK(hipEventSynchronize(e1));
    float ms = 0;
    CHECK(hipEventElapsedTime(&ms, e0, e1));
    ms /= 20;
    std::printf(", {\"kernel\": \"%s\", \"us\": %.1f, \"GBps\": %.1f}",
                kind ? "planes16_two_columns_per_lane" : "planes16_step_order", ms * 1e3,
                pbytes / ms / 1e6);
  }
  std::printf("]}\n");
  CHECK(hipFree(pa));
  CHECK(hipFree(pb));
  return 0;
}
