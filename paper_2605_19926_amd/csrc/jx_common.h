// jx_common.h -- helpers shared by the host translation units.
#pragma once
#include <rocprofiler-sdk-roctx/roctx.h>

#include <string>
#include <vector>

#include "jx.h"
#include "jx_internal.h"

namespace jx {
// A named roctx range for the lifetime of the object: rocprofv3
// --marker-trace shows the library's calls (reset, step, rollout, render,
// serving launches) beside the kernels they enqueue; without a tracer the
// calls are no-ops.
struct TraceRange {
  explicit TraceRange(const char* name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

jx_status set_error(jx_status code, const std::string& msg);
bool validate_cfg(const jx_env_cfg& c, std::string* why);
// Frame format of a configuration (obs_layout * 3 + obs_dtype) and its frame bytes.
int obs_fmt_of(const jx_env_cfg& c);
int64_t frame_bytes(const jx_env_cfg& c);
// Required alignment of frame buffers and strides: the floating formats store
// 8- and 16-byte vectors.
inline int obs_align(int fmt) { return fmt % 3 == 0 ? 4 : 16; }
DevCfg derive_cfg(const jx_env_cfg& c);
Layout make_layout(int n, int n_cfgs, int64_t maps_bytes);
int64_t map_bytes_of(int side);
DevState bind_state(uint8_t* ws, const Layout& L, int n);
void set_uniform(DevState* s, const jx_env_cfg* cfgs, int n_cfgs, const std::vector<int32_t>& idx);
jx_status build_image(int n, const uint64_t* seeds, const jx_env_cfg* cfgs, int n_cfgs,
                      const int32_t* cfg_index, std::vector<uint8_t>* img, Layout* L,
                      std::vector<int64_t>* obs_off, std::vector<int32_t>* idx);
// JX_OK when the state image b (laid out as L) may be loaded into a context of
// n envs with these configurations, else JX_EINVAL with the reason.
jx_status check_state_image(const uint8_t* b, const Layout& L, int n, const std::vector<jx_env_cfg>& cfgs,
                            const std::vector<int32_t>& cfg_idx);
// Thread-local message of the last error (jx_last_error).
extern thread_local std::string g_last_error;
}  // namespace jx
