// Host orderings (plan time); see host_order.cpp.
#pragma once
#include <cstdint>

namespace vecchia {
void order_coord(const double* locs, int64_t D, int64_t* perm);
void order_maxmin(const double* locs, int64_t D, int64_t* perm);
}  // namespace vecchia
