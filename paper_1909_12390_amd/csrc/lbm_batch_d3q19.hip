// Instantiation of the batched D3Q19 kernels (storage x collision x forcing x largest nc).
#include "lbm_batch_dispatch.hpp"

namespace lbmk {
BOps bops_d3q19(int st, int coll, int forc, int ncmax) { return bops_lat<LBM_D3Q19>(st, coll, forc, ncmax); }
}  // namespace lbmk
