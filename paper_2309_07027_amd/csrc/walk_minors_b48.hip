// walk_minors_b48.hip -- leave-one-column-out batch kernel for up to 48 columns.
#include "kernels.hpp"
#include "walk_minors.hpp"

namespace bbfg {

const void* walk_minors_fn_b48() { return reinterpret_cast<const void*>(&walk_minors_batch_kernel<48>); }

}  // namespace bbfg
