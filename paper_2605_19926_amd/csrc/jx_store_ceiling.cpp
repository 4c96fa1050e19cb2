// jx_store_ceiling -- calibration of the HBM write rate that store patterns
// reach on this device, with constant data and no other work, as a ceiling to
// compare the renderer's frame writes against (bench.py runs it and reports
// the figures beside the roofline).  Prints one JSON line of GB/s figures:
//   one_shot_16B_linear   one 16-byte store per thread, blocks in address
//                         order, each block exits after its store (the fastest
//                         pattern found; a plain device fill)
//   one_shot_12B_linear   the same with 12-byte stores
//   one_shot_frame_block  one 12,288-byte frame per 256-thread block
//   env_frames_12B        the renderer's pattern: one wave per env (4096 envs,
//                         8 waves per workgroup) writes its 64x64 RGB frame of
//                         every step as mirrored row pairs of 12-byte lane
//                         stores, 128 steps into 128 frame slots
//   env_frames_84px_12B   the same pattern for 84x84 frames (8192 envs, 21
//                         column groups of 12 bytes, 63 lanes, 3 row pairs per
//                         iteration), 128 steps into 36 slots of 173 MB
// The buffer is 128 x 4096 x 12,288 bytes (6.4 GB, the headline frame ring).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

namespace {

typedef uint32_t u32x3 __attribute__((ext_vector_type(3)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
constexpr int kEnvs = 4096, kFrame = 12288, kSlots = 128, kRow = 192;
constexpr int64_t kSlot = (int64_t)kEnvs * kFrame;
constexpr int64_t kBytes = kSlot * kSlots;
static_assert(kBytes % (16 * 256) == 0 && kBytes % (12 * 256) == 0 && kBytes % kFrame == 0, "sizes");

__global__ __launch_bounds__(256) void one_shot_16(uint8_t* p) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  *(u32x4*)(p + i * 16) = u32x4{0x3C323232u, 0x3C3C3232u, 0x32323C3Cu, 0x3C3C3C32u};
}

__global__ __launch_bounds__(256) void one_shot_12(uint8_t* p) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  *(u32x3*)(p + i * 12) = u32x3{0x3C323232u, 0x3C3C3232u, 0x32323C3Cu};
}

__global__ __launch_bounds__(256) void one_shot_frame(uint8_t* p) {
  uint8_t* f = p + (int64_t)blockIdx.x * kFrame;
  for (int k = 0; k < kFrame / 4096; ++k)
    *(u32x4*)(f + k * 4096 + 16 * threadIdx.x) = u32x4{0x3C323232u, 0x3C3C3232u, 0x32323C3Cu, 0x3C3C3C32u};
}

// lane -> (row distance i = lane / 16, column group cq = lane % 16); each
// iteration stores the row pair at distance i above and below the horizon
__global__ __launch_bounds__(512) void env_frames(uint8_t* p, int steps) {
  const int env = (int)blockIdx.x * 8 + (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
  if (env >= kEnvs) return;
  const u32x3 v{0x3C323232u, 0x3C3C3232u, 0x32323C3Cu};
  const int i0 = lane >> 4, cq = lane & 15;
  for (int t = 0; t < steps; ++t) {
    uint8_t* f = p + (int64_t)(t % kSlots) * kSlot + (int64_t)env * kFrame;
    for (int i = i0; i < 32; i += 4) {
      *(u32x3*)(f + (31 - i) * kRow + 12 * cq) = v;
      *(u32x3*)(f + (32 + i) * kRow + 12 * cq) = v;
    }
  }
}

// The renderer's pattern at W x W frames (W a multiple of 4, W / 4 groups of
// 12 bytes): lane -> (group cq = lane % Q, row distance lane / Q); the wave's
// di * Q lanes cover di = 64 / Q row pairs per iteration.
template <int W>
__global__ __launch_bounds__(512) void env_frames_w(uint8_t* p, int n, int steps, int slots) {
  constexpr int Q = W / 4, di = 64 / Q, H2 = W / 2, row = 3 * W;
  constexpr int64_t frame = (int64_t)row * W;
  const int env = (int)blockIdx.x * 8 + (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
  if (env >= n || lane >= di * Q) return;
  const u32x3 v{0x3C323232u, 0x3C3C3232u, 0x32323C3Cu};
  const int cq = lane % Q, i0 = lane / Q;
  for (int t = 0; t < steps; ++t) {
    uint8_t* f = p + ((int64_t)(t % slots) * n + env) * frame;
    for (int i = i0; i < H2; i += di) {
      *(u32x3*)(f + (int64_t)(H2 - 1 - i) * row + 12 * cq) = v;
      *(u32x3*)(f + (int64_t)(H2 + i) * row + 12 * cq) = v;
    }
  }
}
constexpr int kEnvs84 = 8192, kSlots84 = 36;
static_assert((int64_t)kSlots84 * kEnvs84 * 3 * 84 * 84 <= kBytes, "84x84 ring fits the buffer");

}  // namespace

int main() {
  uint8_t* buf = nullptr;
  if (hipMalloc(&buf, (size_t)kBytes) != hipSuccess) {
    std::fprintf(stderr, "jx_store_ceiling: cannot allocate %lld bytes\n", (long long)kBytes);
    return 1;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return 1;
  const char* names[5] = {"one_shot_16B_linear", "one_shot_12B_linear", "one_shot_frame_block", "env_frames_12B",
                          "env_frames_84px_12B"};
  double best[5] = {0, 0, 0, 0, 0};
  const int reps = 3;
  for (int round = 0; round < 2; ++round) {
    for (int m = 0; m < 5; ++m) {
      auto launch = [&]() {
        switch (m) {
          case 0: hipLaunchKernelGGL(one_shot_16, dim3((unsigned)(kBytes / 16 / 256)), dim3(256), 0, 0, buf); break;
          case 1: hipLaunchKernelGGL(one_shot_12, dim3((unsigned)(kBytes / 12 / 256)), dim3(256), 0, 0, buf); break;
          case 2: hipLaunchKernelGGL(one_shot_frame, dim3((unsigned)(kBytes / kFrame)), dim3(256), 0, 0, buf); break;
          case 3: hipLaunchKernelGGL(env_frames, dim3(kEnvs / 8), dim3(512), 0, 0, buf, kSlots); break;
          default:
            hipLaunchKernelGGL(env_frames_w<84>, dim3(kEnvs84 / 8), dim3(512), 0, 0, buf, kEnvs84, 128, kSlots84);
            break;
        }
      };
      // bytes one launch writes
      const double bytes = m < 4 ? (double)kBytes : 128.0 * kEnvs84 * 3 * 84 * 84;
      launch();
      if (hipDeviceSynchronize() != hipSuccess || hipEventRecord(e0, 0) != hipSuccess) return 1;
      for (int r = 0; r < reps; ++r) launch();
      float ms = 0.f;
      if (hipEventRecord(e1, 0) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess || hipGetLastError() != hipSuccess) {
        std::fprintf(stderr, "jx_store_ceiling: a launch failed\n");
        return 1;
      }
      const double gbs = (double)reps * bytes / (ms * 1e-3) / 1e9;
      if (gbs > best[m]) best[m] = gbs;
    }
  }
  std::printf("{");
  for (int m = 0; m < 5; ++m) std::printf("%s\"%s\": %.1f", m ? ", " : "", names[m], best[m]);
  std::printf("}\n");
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(buf);
  return 0;
}
