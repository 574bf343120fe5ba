// Fused 2D cell kernel, tile height 4.
#define CELL_ROWS 4
#include "cell2d_rows.hpp"
