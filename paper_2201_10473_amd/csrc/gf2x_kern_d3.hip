// gf2x_kern_d3.hip -- kernels of the direct classes with id mod 4 == 3.
#define GF2X_GROUP 3
#define GF2X_GROUP_FN direct_kernels_3
#include "gf2x_kern_direct.hpp"

GF2X_DIRECT_GROUP_BODY()
