// Instantiation of every D2Q9 kernel variant (nc 1..4 x storage x collision x forcing).
#include "lbm_dispatch.hpp"

namespace lbmk {
Ops ops_d2q9(int nc, int st, int coll, int forc) { return ops_lat<LBM_D2Q9>(nc, st, coll, forc); }
AdjOps adj_ops_d2q9(int nc, int st, int coll, int forc) { return adj_ops_lat<LBM_D2Q9>(nc, st, coll, forc); }
}  // namespace lbmk
