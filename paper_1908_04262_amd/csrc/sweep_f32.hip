// Lattice sweep, binary32 and 16-bit-storage instances: multiply-adds may contract into
// fused operations (these instances are held to tolerances, not to bit equality).
#pragma clang fp contract(fast)
#include "sweep_impl.h"

namespace mf {
template void Ops<2, 1>::sweep(Ctx &, hipStream_t);
template void Ops<2, 2>::sweep(Ctx &, hipStream_t);
template void Ops<2, 3>::sweep(Ctx &, hipStream_t);
template void Ops<3, 1>::sweep(Ctx &, hipStream_t);
template void Ops<3, 2>::sweep(Ctx &, hipStream_t);
template void Ops<3, 3>::sweep(Ctx &, hipStream_t);
}  // namespace mf
