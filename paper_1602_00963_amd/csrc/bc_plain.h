// The plain form (one source per launch) replayed from a HIP graph: a
// captured sequence of identical launches takes its sources from a device
// list instead of its launch arguments.
#pragma once
#include "bc_kernels.h"

namespace bcx {

// One per-source launch: the source, the folded sources it represents and
// their subtree term (1-degree reduction), and its score weight.
struct PlainSrc {
  int32_t v;
  int32_t own;
  double tsub;
  double weight;
};

// Device source list: a launch runs srcs[*cursor] and its last step advances
// *cursor, so K captured launches replayed G / K times run G sources in list
// order; a launch that finds the list used up returns before any work.
// srcs == nullptr: the launch runs the source in its PlainArgs.
struct PlainFeed {
  const PlainSrc* srcs;
  int32_t* cursor;
  int32_t nsrc;
};

hipError_t launch_plain_fed(const PlainArgs& a, const PlainFeed& f, bool ext, int grid, int block, hipStream_t st);

}  // namespace bcx
