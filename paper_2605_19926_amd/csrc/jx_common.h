// jx_common.h -- helpers shared by the host translation units.
#pragma once
#include <string>
#include <vector>

#include "jx.h"
#include "jx_internal.h"

namespace jx {
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
}  // namespace jx
