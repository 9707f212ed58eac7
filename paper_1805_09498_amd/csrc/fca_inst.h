// Instantiates every kernel of one (I, J) = (FCA_I, FCA_J) pair and exposes
// its host launchers.  The build compiles one translation unit per pair.
#include "fca_adjoint.h"
#include "fca_em_resident.h"
#include "fca_resident.h"

#define FCA_CAT4_(a, b, c, d) a##b##c##d
#define FCA_CAT4(a, b, c, d) FCA_CAT4_(a, b, c, d)

namespace fca {
const KernelSet* FCA_CAT4(kernel_set_I, FCA_I, _J, FCA_J)() {
  static const KernelSet set = {
      &launch_as_iter_stream<FCA_I, FCA_J>, &launch_as_iter_resident<FCA_I, FCA_J>,
      &as_resident_fits<FCA_I, FCA_J>,      &launch_as_batch_resident<FCA_I, FCA_J>,
      &launch_em_iter<FCA_I, FCA_J>,
      &launch_em_iter_resident<FCA_I, FCA_J>, &em_resident_fits<FCA_I, FCA_J>,
      &launch_as_loglik<FCA_I, FCA_J>,      &launch_em_loglik<FCA_I, FCA_J>,
      &launch_as_wiener<FCA_I, FCA_J>,      &launch_em_wiener<FCA_I, FCA_J>,
      &launch_em_from_as<FCA_I, FCA_J>,     &launch_em_rinv<FCA_I, FCA_J>,
      &launch_as_iter_resident_trace<FCA_I, FCA_J>,
      &launch_adj_iter<FCA_I, FCA_J>,       &launch_adj_seg<FCA_I, FCA_J>,
      &launch_adj_wiener<FCA_I, FCA_J>,
      &launch_check_matrices<FCA_I, FCA_J>};
  return &set;
}
}  // namespace fca
