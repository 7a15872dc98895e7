// Shared host/device definitions of the ptymi library.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>

namespace pty {

// Integer floor and fractional part of a patch's top-left corner.
struct PosInfo {
  int iy, ix;
  float fy, fx;
};

// One object tile and its list of overlapping patches (CSR slice).
struct TileEntry {
  int ty, tx;   // tile origin in object pixels
  int beg, end; // range in the entry list
};

// An entry of a tile's patch list: the patch's slot in the contribution
// buffer, its global position index and a copy of its position (so that a
// tile walk needs one load per patch).
struct alignas(16) PatchRef {
  int slot, j;
  int iy, ix;
  float fy, fx;
  int pad0, pad1;
};

constexpr int kTileH = 16;   // object tile height (rows): one thread walks a column of the tile
constexpr int kTileW = 64;   // object tile width (columns): one wavefront per tile

struct DeviceError : std::runtime_error {
  explicit DeviceError(const std::string& m) : std::runtime_error(m) {}
};
struct NoMemError : std::runtime_error {
  explicit NoMemError(const std::string& m) : std::runtime_error(m) {}
};

inline void hip_check(hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory) throw NoMemError(std::string(what) + ": " + hipGetErrorString(e));
  if (e != hipSuccess) throw DeviceError(std::string(what) + ": " + hipGetErrorString(e));
}

#define PTY_HIP(call) ::pty::hip_check((call), #call)
#define PTY_LAUNCH_CHECK(name) ::pty::hip_check(hipGetLastError(), name)

}  // namespace pty
