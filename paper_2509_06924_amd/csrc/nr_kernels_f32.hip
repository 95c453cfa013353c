// FP32 instantiation of the kernels, shallow buckets (layer product and adjoint in float;
// kz0^2 - 4 pi drho, smearing, chi^2 and gradient accumulation in FP64).
#include "nr_kernels.hpp"

namespace nr {

NR_DEFINE_GRAD_LAUNCHER(launch_grad_shallow, NR_BUCKETS_SHALLOW)

hipError_t launch_forward_f32(int op, bool split, const KernelArgs& a, int n_wu, hipStream_t st) {
  return launch_forward_p<F32>(op, split, a, n_wu, st);
}

hipError_t launch_grad_f32(int bucket, int form, int mode, const KernelArgs& a, int n_wu,
                           hipStream_t st) {
  return launch_grad_shallow<F32>(bucket, form, mode, a, n_wu, st);
}

}  // namespace nr
