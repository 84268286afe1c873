// gf2x_kern_d2.hip -- kernels of the direct classes with id mod 4 == 2.
#define GF2X_GROUP 2
#define GF2X_GROUP_FN direct_kernels_2
#include "gf2x_kern_direct.hpp"

GF2X_DIRECT_GROUP_BODY()
