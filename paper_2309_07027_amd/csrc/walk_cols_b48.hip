// walk_cols_b48.hip -- batch kernel with column multiplicities, up to 48 distinct columns.
#include "kernels.hpp"
#include "walk_batch.hpp"

namespace bbfg {

const void* walk_cols_fn_b48() { return reinterpret_cast<const void*>(&walk_batch_kernel<48, double, true>); }

}  // namespace bbfg
