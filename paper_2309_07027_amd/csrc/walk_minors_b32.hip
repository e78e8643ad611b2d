// walk_minors_b32.hip -- leave-one-column-out batch kernel for up to 32 columns.
#include "kernels.hpp"
#include "walk_minors.hpp"

namespace bbfg {

const void* walk_minors_fn_b32() { return reinterpret_cast<const void*>(&walk_minors_batch_kernel<32>); }

}  // namespace bbfg
