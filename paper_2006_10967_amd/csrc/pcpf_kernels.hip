// Kernels and launchers shared by every (d, p): the launch-table dispatch, the reset and the
// final pass of the FP64 reductions. The (d, p) kernels are templates in
// pcpf_kernels_impl.h, instantiated per dimension and precision in
// pcpf_kernels_{2d,3d}_{f64,f32}.hip.
#include "pcpf_kernels_impl.h"

namespace pcpf {

extern template bool get_launchers_dim<double, 2>(int, Launchers<double>*);
extern template bool get_launchers_dim<double, 3>(int, Launchers<double>*);
extern template bool get_launchers_dim<float, 2>(int, Launchers<float>*);
extern template bool get_launchers_dim<float, 3>(int, Launchers<float>*);

template <typename R>
bool get_launchers(int d, int p, Launchers<R>* L) {
    if (d == 2) return get_launchers_dim<R, 2>(p, L);
    if (d == 3) return get_launchers_dim<R, 3>(p, L);
    return false;
}
template bool get_launchers<double>(int, int, Launchers<double>*);
template bool get_launchers<float>(int, int, Launchers<float>*);

namespace {

__global__ __launch_bounds__(REDUCE_THREADS) void k_reduce_final(const double* partial, int nb,
                                                                double* out) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < nb; i += REDUCE_THREADS) acc += partial[i];
    const double b = block_sum(acc);
    if (threadIdx.x == 0) *out = b;
}

template <typename R>
__global__ void k_reset(const R* phi, R* psi, int64_t n, int mode, double eps_w, double dphi) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (mode == PCPF_RESET_LOGIT) {
        double c = (double)phi[i];
        c = c < dphi ? dphi : (c > 1.0 - dphi ? 1.0 - dphi : c);
        psi[i] = (R)(eps_w * ::log(c / (1.0 - c)));
    } else {
        psi[i] = phi[i] - R(0.5);
    }
}

}  // namespace

template <typename R>
void launch_reset(const R* phi, R* psi, int64_t n, int mode, double eps_w, double delta_phi,
                  hipStream_t s) {
    const unsigned g = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL((k_reset<R>), dim3(g), dim3(256), 0, s, phi, psi, n, mode, eps_w, delta_phi);
}
template void launch_reset<double>(const double*, double*, int64_t, int, double, double, hipStream_t);
template void launch_reset<float>(const float*, float*, int64_t, int, double, double, hipStream_t);

void launch_reduce_final(const double* partial, int nblocks, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(REDUCE_THREADS), 0, s, partial, nblocks, out);
}

}  // namespace pcpf
