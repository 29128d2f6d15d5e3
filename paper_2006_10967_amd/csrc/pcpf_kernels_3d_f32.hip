// The 3D kernels in float: one translation unit per dimension and precision, so that the
// instantiations compile in parallel.
#include "pcpf_kernels_impl.h"

namespace pcpf {
template bool get_launchers_dim<float, 3>(int, Launchers<float>*);
}  // namespace pcpf
