// gf2x_kern_d1.hip -- kernels of the direct classes with id mod 4 == 1.
#define GF2X_GROUP 1
#define GF2X_GROUP_FN direct_kernels_1
#include "gf2x_kern_direct.hpp"

GF2X_DIRECT_GROUP_BODY()
