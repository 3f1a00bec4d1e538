// Fused sweep shapes for IEEE binary32 storage (16-byte vector = 4 elements):
// (workgroup, lanes per row, chunks, rows per step, steps in flight + 1); 16 or 32 lanes per row
// sweep four or two short rows per wavefront.
// Every shape listed compiles without register spills.
#define MODAP_DT 1
#define MODAP_SHAPES                                                                              \
    MODAP_SHAPE(256, 16, 1, 1, 2), MODAP_SHAPE(256, 16, 2, 1, 2), MODAP_SHAPE(256, 16, 4, 1, 2),          \
    MODAP_SHAPE(256, 32, 2, 1, 2), MODAP_SHAPE(256, 32, 4, 1, 2),                                         \
    MODAP_SHAPE(256, 64, 1, 1, 2), MODAP_SHAPE(256, 64, 2, 1, 2), MODAP_SHAPE(256, 64, 4, 1, 2),          \
    MODAP_SHAPE(256, 64, 1, 2, 2), MODAP_SHAPE(256, 64, 2, 2, 2), MODAP_SHAPE(256, 64, 4, 2, 2),          \
    MODAP_SHAPE(256, 256, 2, 1, 2), MODAP_SHAPE(256, 256, 4, 1, 2), MODAP_SHAPE(256, 256, 8, 1, 2),       \
    MODAP_SHAPE(256, 256, 2, 2, 2), MODAP_SHAPE(256, 256, 4, 2, 2), MODAP_SHAPE(256, 256, 2, 4, 2),       \
    MODAP_SHAPE(512, 512, 2, 1, 2), MODAP_SHAPE(512, 512, 4, 1, 2), MODAP_SHAPE(512, 512, 8, 1, 2),       \
    MODAP_SHAPE(512, 512, 2, 2, 2), MODAP_SHAPE(512, 512, 4, 2, 2), MODAP_SHAPE(512, 512, 2, 4, 2),       \
    MODAP_SHAPE(1024, 1024, 2, 1, 2), MODAP_SHAPE(512, 256, 8, 1, 2), MODAP_SHAPE(512, 256, 4, 1, 2),     \
    MODAP_SHAPE(512, 512, 4, 1, 3), MODAP_SHAPE(512, 512, 4, 1, 4),                                      \
    MODAP_SHAPE(1024, 1024, 2, 1, 3)
// split-row form: 256 lanes x 8 chunks per column tile
#define MODAP_SPLIT_C 8
#include "sweep_inst.inc"
