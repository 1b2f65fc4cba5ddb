// Lattice sweep, binary32 instance: multiply-adds may contract into fused operations
// (this instance is held to tolerances, not to bit equality).
#pragma clang fp contract(fast)
#include "sweep_impl.h"

namespace mf {
template bool Ops<2, 1>::sweep_bulk_auto(Ctx &, hipStream_t);
template void Ops<2, 1>::sweep_interface(Ctx &, hipStream_t);
template void Ops<2, 1>::sweep_cells(Ctx &, hipStream_t);
template void Ops<2, 1>::sweep_multi(const MStep &, unsigned, bool, bool, int, hipStream_t);
template void Ops<2, 1>::bulk_multi(const MStep &, int, bool, hipStream_t);
template bool Ops<2, 1>::sweep_bulk(Ctx &, hipStream_t, int);
template bool Ops<3, 1>::sweep_bulk_auto(Ctx &, hipStream_t);
template void Ops<3, 1>::sweep_interface(Ctx &, hipStream_t);
template void Ops<3, 1>::sweep_cells(Ctx &, hipStream_t);
template void Ops<3, 1>::sweep_multi(const MStep &, unsigned, bool, bool, int, hipStream_t);
template void Ops<3, 1>::bulk_multi(const MStep &, int, bool, hipStream_t);
template bool Ops<3, 1>::sweep_bulk(Ctx &, hipStream_t, int);
}  // namespace mf
