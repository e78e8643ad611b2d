// walk_minors_b16.hip -- leave-one-column-out batch kernel for up to 16 columns.
#include "kernels.hpp"
#include "walk_minors.hpp"

namespace bbfg {

const void* walk_minors_fn_b16() { return reinterpret_cast<const void*>(&walk_minors_batch_kernel<16>); }

}  // namespace bbfg
