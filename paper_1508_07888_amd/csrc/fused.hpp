// fused.hpp -- transport + chemistry in one pass over HBM.
#pragma once

#include "kernels.hpp"

namespace emma {

inline bool fused_supported(const Grid &) { return false; }

template <int G, typename S, bool DIAG>
inline int launch_fused(hipStream_t, const S *, const S *, S *, S *, double *, double *, const double *,
                        const Grid &, const SrcTable &, const GroupConsts &, const ChemParams &, double,
                        unsigned long long *) {
    return -1;
}

}  // namespace emma
