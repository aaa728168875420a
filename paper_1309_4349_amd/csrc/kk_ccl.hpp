// kk_ccl.hpp -- cluster labelling of many square lattices in one set of
// launches (the batch engine's histograms).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kk_kernels.hpp"

namespace kk {

// One square lattice of a labelling launch: its current buffer, layout and
// side, and its labelling buffers (CclBuffers of its handle).
struct CclRep {
  const void* lat;
  int layout, L;
  CclBuffers b;
};

// Label species on every lattice of the device table d_reps (nreps entries,
// the largest of max_sites sites), count, build each one's histogram, and
// copy each result block (histogram, large-size count, first large sizes;
// `words` words) into row i of `stage`.
hipError_t launch_ccl_many(const CclRep* d_reps, int nreps, size_t max_sites, int species, uint32_t* stage,
                           uint32_t words, hipStream_t stream);

}  // namespace kk
