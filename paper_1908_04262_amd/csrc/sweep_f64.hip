// Lattice sweep, binary64 instance: compiled without floating-point contraction so that
// every operation rounds as the method's reference arithmetic prescribes.
#include "sweep_impl.h"

namespace mf {
template void Ops<2, 0>::sweep(Ctx &, hipStream_t, hipEvent_t, hipEvent_t, void (*)(void *), void *);
template bool Ops<2, 0>::sweep_bulk(Ctx &, hipStream_t, int);
template void Ops<3, 0>::sweep(Ctx &, hipStream_t, hipEvent_t, hipEvent_t, void (*)(void *), void *);
template bool Ops<3, 0>::sweep_bulk(Ctx &, hipStream_t, int);
}  // namespace mf
