// The clip-table kernels (one launch over a batch of mixed K) of the family bounded by K <= 8.
#define GID_TABLE_KB 8
#include "gid_kernels_table.inc"
