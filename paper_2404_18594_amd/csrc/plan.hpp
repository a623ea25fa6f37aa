// What the batch code (host_batch.cpp) reads of a plan, defined in host.cpp.
#pragma once

#include <string>

#include "../../include/cdtwa.h"
#include "common.hpp"

namespace cdtwa {

struct PlanLayout {
  size_t state_bytes, field_bytes;
  int dtype, path;
  const int* legs;   // fused paths: [nc][4][4] neighbour legs (device)
  int wide;          // fused path built for three workgroups per CU
  int spin_limit;    // polls a fused kernel's neighbour wait may take
};
bool plan_layout(cdtwa_plan plan, PlanLayout* out);
const Geom* plan_geom(cdtwa_plan plan);
cdtwa_status set_error(cdtwa_status st, const std::string& msg);

}  // namespace cdtwa
