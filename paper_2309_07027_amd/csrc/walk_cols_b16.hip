// walk_cols_b16.hip -- batch kernel with column multiplicities, up to 16 distinct columns.
#include "kernels.hpp"
#include "walk_batch.hpp"

namespace bbfg {

const void* walk_cols_fn_b16() { return reinterpret_cast<const void*>(&walk_batch_kernel<16, double, true>); }

}  // namespace bbfg
