// Lattice sweep, 16-bit-storage instances (binary16 / bfloat16 population offsets,
// binary32 arithmetic): multiply-adds may contract into fused operations (these
// instances are held to tolerances, not to bit equality).
#pragma clang fp contract(fast)
#include "sweep_impl.h"

namespace mf {
template bool Ops<2, 2>::sweep_bulk_auto(Ctx &, hipStream_t);
template void Ops<2, 2>::sweep_interface(Ctx &, hipStream_t);
template void Ops<2, 2>::sweep_cells(Ctx &, hipStream_t);
template void Ops<2, 2>::sweep_multi(const MStep &, unsigned, bool, bool, int, hipStream_t);
template void Ops<2, 2>::bulk_multi(const MStep &, int, bool, hipStream_t);
template bool Ops<2, 2>::sweep_bulk(Ctx &, hipStream_t, int);
template bool Ops<2, 3>::sweep_bulk_auto(Ctx &, hipStream_t);
template void Ops<2, 3>::sweep_interface(Ctx &, hipStream_t);
template void Ops<2, 3>::sweep_cells(Ctx &, hipStream_t);
template void Ops<2, 3>::sweep_multi(const MStep &, unsigned, bool, bool, int, hipStream_t);
template void Ops<2, 3>::bulk_multi(const MStep &, int, bool, hipStream_t);
template bool Ops<2, 3>::sweep_bulk(Ctx &, hipStream_t, int);
template bool Ops<2, 4>::sweep_bulk_auto(Ctx &, hipStream_t);
template void Ops<2, 4>::sweep_interface(Ctx &, hipStream_t);
template void Ops<2, 4>::sweep_cells(Ctx &, hipStream_t);
template void Ops<2, 4>::sweep_multi(const MStep &, unsigned, bool, bool, int, hipStream_t);
template void Ops<2, 4>::bulk_multi(const MStep &, int, bool, hipStream_t);
template bool Ops<2, 4>::sweep_bulk(Ctx &, hipStream_t, int);
template bool Ops<3, 2>::sweep_bulk_auto(Ctx &, hipStream_t);
template void Ops<3, 2>::sweep_interface(Ctx &, hipStream_t);
template void Ops<3, 2>::sweep_cells(Ctx &, hipStream_t);
template void Ops<3, 2>::sweep_multi(const MStep &, unsigned, bool, bool, int, hipStream_t);
template void Ops<3, 2>::bulk_multi(const MStep &, int, bool, hipStream_t);
template bool Ops<3, 2>::sweep_bulk(Ctx &, hipStream_t, int);
template bool Ops<3, 3>::sweep_bulk_auto(Ctx &, hipStream_t);
template void Ops<3, 3>::sweep_interface(Ctx &, hipStream_t);
template void Ops<3, 3>::sweep_cells(Ctx &, hipStream_t);
template void Ops<3, 3>::sweep_multi(const MStep &, unsigned, bool, bool, int, hipStream_t);
template void Ops<3, 3>::bulk_multi(const MStep &, int, bool, hipStream_t);
template bool Ops<3, 3>::sweep_bulk(Ctx &, hipStream_t, int);
template bool Ops<3, 4>::sweep_bulk_auto(Ctx &, hipStream_t);
template void Ops<3, 4>::sweep_interface(Ctx &, hipStream_t);
template void Ops<3, 4>::sweep_cells(Ctx &, hipStream_t);
template void Ops<3, 4>::sweep_multi(const MStep &, unsigned, bool, bool, int, hipStream_t);
template void Ops<3, 4>::bulk_multi(const MStep &, int, bool, hipStream_t);
template bool Ops<3, 4>::sweep_bulk(Ctx &, hipStream_t, int);
}  // namespace mf
