// walk_minors_b30.hip -- leave-one-column-out batch kernel for up to 30 columns.
#include "kernels.hpp"
#include "walk_minors.hpp"

namespace bbfg {

const void* walk_minors_fn_b30() { return reinterpret_cast<const void*>(&walk_minors_batch_kernel<30>); }

}  // namespace bbfg
