// The clip-table kernels (one launch over a batch of mixed K) of the family bounded by K <= 12.
#define GID_TABLE_KB 12
#include "gid_kernels_table.inc"
