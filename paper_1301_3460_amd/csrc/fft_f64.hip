// FFT pass kernels instantiated for double.
#include "fft_kernels.hpp"

namespace lgf {

template size_t fft_xy_lds_bytes<double>(const geom &);
template hipError_t launch_fft_xy<double>(const geom &, void *, int, const void *,
                                          const dev_status *, hipStream_t);
template zt_plan plan_zt<double>(const geom &, size_t);
template void fft_set_max_lds<double>(const geom &, const zt_plan &);
template hipError_t launch_fft_zt<double>(const geom &, void *, int, const void *, const double *,
                                          double, const zt_plan &, const dev_status *, hipStream_t);

}  // namespace lgf
