// FP32 instances of the 2D wave-strip march kernels (strip_march.h).
#include "strip_march.h"

namespace fas {

template void strip_pre<float>(const fas_grid*, int, const Coef&, int, int, const void*, const void*, void*, void*, void*,
                             void*);
template void strip_post<float>(const fas_grid*, int, const Coef&, int, int, const void*, const void*, const void*, void*,
                              double*);
template int strip_waves_per_cu<float>(int);

}  // namespace fas
