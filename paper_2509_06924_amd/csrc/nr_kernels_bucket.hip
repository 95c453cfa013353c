// Gradient kernels of one deep layer-count bucket in one precision.  The
// build compiles this file once per (precision, bucket) of NR_BUCKETS_DEEP
// with -DNR_PREC=F64|F32 -DNR_BUCKET_LMAX=<layers>, so the large unrolled
// kernels build in parallel.
#include "nr_kernels.hpp"

#if !defined(NR_PREC) || !defined(NR_BUCKET_LMAX)
#error "compile with -DNR_PREC=F64|F32 and -DNR_BUCKET_LMAX=<layers>"
#endif

namespace nr {

hipError_t NR_DEEP_LAUNCHER(NR_PREC, NR_BUCKET_LMAX)(int form, int mode, const KernelArgs& a,
                                                     int n_wu, hipStream_t st) {
  using P = NR_PREC;
  constexpr int LM = NR_BUCKET_LMAX;
  if (n_wu <= 0) return hipSuccess;
  NR_FORMS(LM)
  return hipGetLastError();
}

}  // namespace nr
