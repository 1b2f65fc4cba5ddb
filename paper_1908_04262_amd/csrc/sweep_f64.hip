// Lattice sweep, binary64 instance: compiled without floating-point contraction so that
// every operation rounds as the method's reference arithmetic prescribes.
#include "sweep_impl.h"

namespace mf {
template bool Ops<2, 0>::sweep_bulk_auto(Ctx &, hipStream_t);
template void Ops<2, 0>::sweep_interface(Ctx &, hipStream_t);
template void Ops<2, 0>::sweep_cells(Ctx &, hipStream_t);
template void Ops<2, 0>::sweep_multi(const MStep &, unsigned, bool, bool, int, hipStream_t);
template void Ops<2, 0>::bulk_multi(const MStep &, int, bool, hipStream_t);
template bool Ops<2, 0>::sweep_bulk(Ctx &, hipStream_t, int);
template bool Ops<3, 0>::sweep_bulk_auto(Ctx &, hipStream_t);
template void Ops<3, 0>::sweep_interface(Ctx &, hipStream_t);
template void Ops<3, 0>::sweep_cells(Ctx &, hipStream_t);
template void Ops<3, 0>::sweep_multi(const MStep &, unsigned, bool, bool, int, hipStream_t);
template void Ops<3, 0>::bulk_multi(const MStep &, int, bool, hipStream_t);
template bool Ops<3, 0>::sweep_bulk(Ctx &, hipStream_t, int);
}  // namespace mf
