// walk_cols_b24.hip -- batch kernel with column multiplicities, up to 24 distinct columns.
#include "kernels.hpp"
#include "walk_batch.hpp"

namespace bbfg {

const void* walk_cols_fn_b24() { return reinterpret_cast<const void*>(&walk_batch_kernel<24, double, true>); }

}  // namespace bbfg
