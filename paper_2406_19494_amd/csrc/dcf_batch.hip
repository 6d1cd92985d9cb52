// dcf_batch.hip -- batched multi-solve stepping for the serving loop
// (placeholder; filled in with the request scheduler).
#include "dcf_kernels.hpp"
