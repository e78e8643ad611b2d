// walk_cols_b32.hip -- batch kernel with column multiplicities, up to 32 distinct columns.
#include "kernels.hpp"
#include "walk_batch.hpp"

namespace bbfg {

const void* walk_cols_fn_b32() { return reinterpret_cast<const void*>(&walk_batch_kernel<32, double, true>); }

}  // namespace bbfg
