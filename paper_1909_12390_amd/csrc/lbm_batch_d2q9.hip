// Instantiation of the batched D2Q9 kernels (storage x collision x forcing x largest nc).
#include "lbm_batch_dispatch.hpp"

namespace lbmk {
BOps bops_d2q9(int st, int coll, int forc, int ncmax) { return bops_lat<LBM_D2Q9>(st, coll, forc, ncmax); }
}  // namespace lbmk
