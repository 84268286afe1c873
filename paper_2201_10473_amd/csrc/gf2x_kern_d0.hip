// gf2x_kern_d0.hip -- kernels of the direct classes with id mod 4 == 0.
#define GF2X_GROUP 0
#define GF2X_GROUP_FN direct_kernels_0
#include "gf2x_kern_direct.hpp"

GF2X_DIRECT_GROUP_BODY()
