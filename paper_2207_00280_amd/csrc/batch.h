// Internal interface between the C ABI and the batched (many-patch) path.
#pragma once

#include "../../include/igafem.h"
#include "common.h"

namespace igaf {
const PatchDev& plan_dev(const igaf_plan* p);
int plan_degree(const igaf_plan* p);
bool plan_hot_supported(const igaf_plan* p);
igaf_status set_error(igaf_status st, const char* msg);
}  // namespace igaf
