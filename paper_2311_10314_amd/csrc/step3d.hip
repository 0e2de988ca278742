// 3D step kernels (D3Q15 phase sets, D3Q19 flow set).
#include <hip/hip_runtime.h>

#include "coef.hpp"
#include "kernels.hpp"

namespace ddcc {

bool have_3d() { return false; }

template <class S, class R>
hipError_t launch_3d(int, int, const Coef<R>&, const Bufs<S>&, int, int,
                     hipStream_t) {
  return hipErrorNotSupported;
}

template hipError_t launch_3d<double, double>(int, int, const Coef<double>&,
                                              const Bufs<double>&, int, int,
                                              hipStream_t);
template hipError_t launch_3d<float, float>(int, int, const Coef<float>&,
                                            const Bufs<float>&, int, int,
                                            hipStream_t);

}  // namespace ddcc
