// Instantiation of every D3Q19 kernel variant (nc 1..4 x storage x collision x forcing).
#include "lbm_dispatch.hpp"

namespace lbmk {
Ops ops_d3q19(int nc, int st, int coll, int forc) { return ops_lat<LBM_D3Q19>(nc, st, coll, forc); }
AdjOps adj_ops_d3q19(int nc, int st, int coll, int forc) { return adj_ops_lat<LBM_D3Q19>(nc, st, coll, forc); }
}  // namespace lbmk
