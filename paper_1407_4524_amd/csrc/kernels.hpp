// Launchers of the HIP kernels (internal interface of the library).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "geom.hpp"
#include "lattice.hpp"

namespace lbm {

struct BulkShape {
  int nbx, nrows, nplanes, nblocks;
};
BulkShape bulk_shape(const Geom& g, int span);

// stream-collide launch shape: threads per block, nodes per thread,
// non-temporal stores, XCD-aware block order
struct BulkConfig {
  int block, cells_per_thread, nontemporal, remap;
};
BulkConfig bulk_config(int lat, int st, size_t footprint);

hipError_t launch_stream_collide(int lat, int st, int eq, const void* A, void* B, const Geom& g, const Phys& ph,
                                 hipStream_t s, const BulkConfig* cfg = nullptr);
hipError_t launch_init(int lat, int st, int eq, void* A, uint8_t* mask, const Geom& g, const Phys& ph,
                       const double* rho, const double* u, hipStream_t s);
hipError_t launch_links(int lat, int st, int eq, void* A, const Link* links, int n_host, const int* n_dev,
                        int grid, const double* pose, int bc, const uint8_t* mask, const Geom& g, const Phys& ph,
                        double* partials, unsigned* counter, double* rec, hipStream_t s);
hipError_t launch_body_advance(int lat, int st, int eq, void* B, uint8_t* mask, uint8_t* mask_next, Link* links,
                               int* n_links, int cap, const double* pose, const BodyShape& bs, int bc, int body,
                               int mode, const Geom& g, const Phys& ph, double* rec_t, double* rec_t1, int* err,
                               hipStream_t s, int64_t region_cells, int64_t region_rows);

}  // namespace lbm
