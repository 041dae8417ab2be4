// DP kernel instantiations with 4 protein column(s) per lane.
#include "mpg_dp.h"

namespace mpg {

hipError_t launch_dp_k4(hipStream_t s, int ncu, bool tb, const DevParams& P,
                        const PairJob* jobs, const int2* items, int nitems, int* qhead,
                        void* pst, int* prog, const uint8_t* prot, const uint8_t* desc,
                        int2* bnd, uint8_t* tbbuf, const DpSink& sink) {
    return dev::launch_dp_k<4, false>(s, ncu, tb, P, jobs, items, nitems, qhead,
                                    (dev::PairState*)pst, prog, prot, desc, bnd, tbbuf, sink);
}

}  // namespace mpg
