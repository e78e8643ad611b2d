// walk_minors_b24.hip -- leave-one-column-out batch kernel for up to 24 columns.
#include "kernels.hpp"
#include "walk_minors.hpp"

namespace bbfg {

const void* walk_minors_fn_b24() { return reinterpret_cast<const void*>(&walk_minors_batch_kernel<24>); }

}  // namespace bbfg
