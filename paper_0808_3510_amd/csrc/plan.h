// Host plan object behind the opaque pat_plan handle.
#pragma once

#include <cstddef>
#include <string>
#include <vector>

#include "../../include/pat.h"
#include "pat_internal.h"

struct pat_plan {
  pat_geometry g;          // as given, alpha resolved
  int prec = 0;            // pat_precision
  pat::Inst inst;          // host copy of the device descriptor
  std::vector<unsigned char> blob;  // host image of the device table buffer
  size_t off_desc = 0, off_tw = 0, off_perm = 0, off_sn = 0, off_poly = 0, off_cut = 0;
  size_t table_bytes = 0, ws_bytes = 0;
  void* table_dev = nullptr;
  bool uploaded = false;
  bool fusable = false;    // the fused line kernels fit this geometry and precision
  bool spread_ok = false;  // the spreading lists of a depth line fit in LDS (R^T, A)
  bool timing = false;
  void* timer = nullptr;   // owned by the ABI layer
  void* fork = nullptr;    // streams of the batched calls led by this plan (ABI layer)
};

namespace pat {

// Builds the plan (host only).  Returns PAT_OK or an error with a message.
pat_status build_plan(const pat_geometry& g, pat_plan* p, std::string* err);

// Fills the device addresses in the descriptor once the table buffer is known
// and writes the descriptor into the blob.
void bind_table(pat_plan* p, void* table_dev);

// Bytes per complex element and per grid element for a precision.
size_t complex_bytes(int prec);
size_t grid_bytes(int prec);

// Modified Bessel function I0(z) e^{-z} by its power series (z >= 0).
double bessel_i0e(double z);

}  // namespace pat
