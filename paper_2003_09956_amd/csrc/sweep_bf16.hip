// Fused sweep shapes for bfloat16 storage (16-byte vector = 8 elements):
// (workgroup, lanes per row, chunks, rows per step, steps in flight + 1); 16 or 32 lanes per row
// sweep four or two short rows per wavefront.
// Every shape listed compiles without register spills.
#define MODAP_DT 2
#define MODAP_SHAPES                                                                              \
    MODAP_SHAPE(256, 16, 1, 1, 2), MODAP_SHAPE(256, 16, 2, 1, 2), MODAP_SHAPE(256, 16, 4, 1, 2),          \
    MODAP_SHAPE(256, 32, 2, 1, 2),                                                                         \
    MODAP_SHAPE(256, 64, 1, 1, 2), MODAP_SHAPE(256, 64, 2, 1, 2), MODAP_SHAPE(256, 64, 4, 1, 2),          \
    MODAP_SHAPE(256, 64, 1, 2, 2), MODAP_SHAPE(256, 64, 2, 2, 2),                                         \
    MODAP_SHAPE(256, 256, 2, 1, 2), MODAP_SHAPE(256, 256, 4, 1, 2), MODAP_SHAPE(256, 256, 2, 2, 2),       \
    MODAP_SHAPE(512, 512, 2, 1, 2), MODAP_SHAPE(512, 512, 4, 1, 2), MODAP_SHAPE(512, 512, 2, 2, 2),       \
    MODAP_SHAPE(1024, 1024, 1, 1, 2), MODAP_SHAPE(1024, 1024, 1, 1, 4),                                   \
    MODAP_SHAPE(256, 256, 4, 1, 3), MODAP_SHAPE(512, 512, 2, 2, 3), MODAP_SHAPE(512, 512, 4, 1, 3)
// split-row form: 256 lanes x 4 chunks per column tile
#define MODAP_SPLIT_C 4
#include "sweep_inst.inc"
