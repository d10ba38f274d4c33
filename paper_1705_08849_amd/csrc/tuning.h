// Tile-shape selection for the stencil launches.  Defaults come from the grid
// shape; the autotuner (tuning.hip) measures the compiled shapes on the device
// and records the fastest per (grid shape, dtype) in a process-wide table
// that can be saved to / loaded from a JSON cache.
#pragma once

#include <cmath>

#include "fit_internal.h"
#include "stencil.h"

namespace fit {

// Makes `dev` current for the scope of a call and restores the previous one.
struct DeviceScope {
  int prev = -1;
  explicit DeviceScope(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceScope() {
    int cur;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

// Default: 64x4 node tiles; z-chunks sized so that the launch has at least
// ~4 workgroups per CU of the 256-CU device while each chunk stays >= 8
// planes deep (the warm-up plane costs 1/ZC extra reads).
TileShape default_tile(const GridView& g, int dtype);
// Tuned shape if one is recorded for this grid shape and dtype, else the default.
TileShape tile_for(const fit_grid* g, int dtype);

}  // namespace fit
