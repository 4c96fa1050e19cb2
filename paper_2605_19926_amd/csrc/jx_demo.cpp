// jx_demo.cpp -- a C++ caller of the C-ABI with no Python or PyTorch: device
// memory from hipMalloc, one context on the default stream, a reset, one fused
// rollout, results copied back.  It prints a line of figures that the test
// suite reproduces through the Python binding.
//
//   jx_demo [n_envs] [steps]        (defaults 256, 128)
//
// Workload: 16x16 mazes with 10% loops, goal billboard, 6 actions, episode cap
// 512, 64x64 RGB frames; env i has seed (7 << 32) | i; the action of env i at
// step t is splitmix64(t * n_envs + i + 1) mod 6.
#include <hip/hip_runtime_api.h>

#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "jx.h"

namespace {

uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

// FNV-1a, 64-bit
uint64_t fnv1a(const uint8_t* p, size_t n) {
  uint64_t h = 0xCBF29CE484222325ull;
  for (size_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= 0x100000001B3ull;
  }
  return h;
}

int fail(const char* what, int code) {
  std::fprintf(stderr, "jx_demo: %s failed (%d): %s\n", what, code, jx_last_error());
  return 1;
}

}  // namespace

int main(int argc, char** argv) {
  const int n = argc > 1 ? std::atoi(argv[1]) : 256;
  const int T = argc > 2 ? std::atoi(argv[2]) : 128;
  if (n < 1 || n > (1 << 20) || T < 1 || T > 4096) {
    std::fprintf(stderr, "usage: jx_demo [n_envs 1..1048576] [steps 1..4096]\n");
    return 2;
  }
  if (jx_abi_version() != JX_ABI_VERSION) {
    std::fprintf(stderr, "jx_demo: library ABI %d, header %d\n", jx_abi_version(), JX_ABI_VERSION);
    return 1;
  }
  jx_env_cfg cfg{};
  cfg.side = 16;
  cfg.n_colors = 8;
  cfg.loop_frac = 0.1f;
  cfg.key_door = 0;
  cfg.goal_sprite = 1;
  cfg.max_decor = 0;
  cfg.obs_h = 64;
  cfg.obs_w = 64;
  cfg.fov_deg = 60.f;
  cfg.n_actions = 6;
  cfg.episode_cap = 512;
  cfg.move = 0.1f;
  cfg.turn = (float)(M_PI / 16.0);
  cfg.pickup_radius = 0.3f;
  cfg.r_goal = 1.f;
  cfg.r_key = 0.5f;
  cfg.shade_levels = 0;
  cfg.shade_dist = 8.f;
  cfg.ascii_map = nullptr;
  cfg.obs_layout = JX_OBS_NHWC;
  cfg.obs_dtype = JX_OBS_U8;

  std::vector<uint64_t> seeds(n);
  for (int i = 0; i < n; ++i) seeds[i] = (7ull << 32) | (uint64_t)i;
  std::vector<uint8_t> acts((size_t)T * n);
  for (int t = 0; t < T; ++t)
    for (int i = 0; i < n; ++i)
      acts[(size_t)t * n + i] = (uint8_t)(splitmix64((uint64_t)t * n + i + 1) % 6);

  const size_t ws_bytes = jx_workspace_bytes(n, &cfg, 1, nullptr);
  if (ws_bytes == 0) return fail("jx_workspace_bytes", -1);
  void* ws = nullptr;
  if (hipMalloc(&ws, ws_bytes) != hipSuccess) return fail("hipMalloc(workspace)", -1);
  jx_ctx* ctx = nullptr;
  jx_status st = jx_create(&ctx, 0, nullptr, ws, ws_bytes);
  if (st) return fail("jx_create", st);
  st = jx_reset(ctx, n, seeds.data(), &cfg, 1, nullptr, nullptr);
  if (st) return fail("jx_reset", st);
  const int64_t ob = jx_obs_bytes(ctx);
  uint8_t *d_act = nullptr, *d_obs = nullptr, *d_done = nullptr;
  float* d_rew = nullptr;
  if (hipMalloc((void**)&d_act, acts.size()) != hipSuccess ||
      hipMalloc((void**)&d_obs, (size_t)ob * T) != hipSuccess ||
      hipMalloc((void**)&d_rew, sizeof(float) * (size_t)T * n) != hipSuccess ||
      hipMalloc((void**)&d_done, (size_t)T * n) != hipSuccess)
    return fail("hipMalloc(buffers)", -1);
  if (hipMemcpy(d_act, acts.data(), acts.size(), hipMemcpyHostToDevice) != hipSuccess)
    return fail("hipMemcpy(actions)", -1);

  const auto t0 = std::chrono::steady_clock::now();
  st = jx_rollout(ctx, T, d_act, d_obs, ob, d_rew, d_done, nullptr, JX_ROLLOUT_FUSED);
  if (st) return fail("jx_rollout", st);
  st = jx_sync(ctx);
  if (st) return fail("jx_sync", st);
  const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();

  std::vector<float> rew((size_t)T * n);
  std::vector<uint8_t> done((size_t)T * n), last((size_t)ob);
  if (hipMemcpy(rew.data(), d_rew, sizeof(float) * rew.size(), hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(done.data(), d_done, done.size(), hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(last.data(), d_obs + (size_t)ob * (T - 1), (size_t)ob, hipMemcpyDeviceToHost) != hipSuccess)
    return fail("hipMemcpy(results)", -1);
  double rsum = 0.0;
  long dones = 0;
  for (size_t k = 0; k < rew.size(); ++k) {
    rsum += rew[k];
    dones += done[k];
  }
  std::printf("envs %d steps %d reward_sum %.1f dones %ld last_frames_fnv1a %016llx env_steps_per_s %.3e\n", n, T,
              rsum, dones, (unsigned long long)fnv1a(last.data(), last.size()), (double)n * T / sec);
  jx_destroy(ctx);
  hipFree(d_act);
  hipFree(d_obs);
  hipFree(d_rew);
  hipFree(d_done);
  hipFree(ws);
  return 0;
}
