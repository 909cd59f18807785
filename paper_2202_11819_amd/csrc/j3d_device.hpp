// j3d_device.hpp -- small HIP runtime helpers shared by the solver, batch and pool.
#pragma once

#include <hip/hip_runtime_api.h>

#include "j3d_host.hpp"

namespace j3d {

// EDEVICE with the HIP error text when `e` is not hipSuccess.
j3d_status hip_status(hipError_t e, const char *what);
inline j3d_status hip_status(int e, const char *what) { return hip_status((hipError_t)e, what); }

// The current device must be a gfx950; fills its compute-unit count.
j3d_status require_device(int *device, int *cus);

// Upload the block, problem and per-axis map tables of a plan to the arena.
j3d_status upload_tables(const Plan &plan, char *arena, hipStream_t stream);

// Upload a tile list to the arena's tile table.
j3d_status upload_tiles(const Plan &plan, const std::vector<Tile> &tiles, char *arena,
                        hipStream_t stream);

// Seeded initialisation of every problem of a plan (interior of parity 0,
// halo storage of both parities).
j3d_status init_fields(const Plan &plan, char *arena, hipStream_t stream);

// Pack, exchange and unpack (Fig. 1 / Fig. 3) of parity `parity` for blocks
// [b0, b1): afterwards every interior-face halo equals the neighbour's face.
j3d_status refresh_halos(const Plan &plan, char *arena, int32_t b0, int32_t b1, int parity,
                         hipStream_t stream);

// Dense interior of problem `i` to/from `dense` (device or host), parity `parity`.
j3d_status copy_dense(const Plan &plan, char *arena, int32_t i, int parity, double *dense,
                      int dense_on_device, bool to_dense, hipStream_t stream);

}  // namespace j3d
