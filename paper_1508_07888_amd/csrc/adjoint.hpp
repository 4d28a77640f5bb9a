// adjoint.hpp -- reverse-mode derivative of the radiation step.
#pragma once

#include "kernels.hpp"
#include "../../include/emma_rt.h"

namespace emma {

struct AdjointScratch {
    void *tape;
    int64_t bytes;
};

struct AdjointCall {
    hipStream_t stream;
    Grid grid;
    GroupConsts gc;
    emma_rt_config cfg;
    double dt;
    int n_steps;
    const uint32_t *mask;
    const int64_t *sorted_cell;
    const double *S;
    const int32_t *sorted_idx;
    int n_src;
    void *Ns, *Fs;
    unsigned long long *cnt;
};

inline int64_t adjoint_scratch_bytes(const emma_rt_config &) { return 0; }
inline int adjoint_alloc(AdjointScratch &a, const emma_rt_config &) {
    a.tape = nullptr;
    a.bytes = 0;
    return 0;
}
inline void adjoint_release(AdjointScratch &a) {
    if (a.tape) (void)hipFree(a.tape);
    a.tape = nullptr;
}

template <int G, typename S>
inline int adjoint_run(AdjointScratch &, const AdjointCall &, const S *, const S *, const double *,
                       const double *, const double *, const double *, S *, S *, double *, double *,
                       double *, double *) {
    return -1;
}

}  // namespace emma
