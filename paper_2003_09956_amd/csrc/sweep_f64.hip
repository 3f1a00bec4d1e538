// Fused sweep shapes for IEEE binary64 storage (16-byte vector = 2 elements).
#define MODAP_DT 0
#define MODAP_SHAPES                                                                     \
    MODAP_SHAPE(256, 64, 1), MODAP_SHAPE(256, 64, 2), MODAP_SHAPE(256, 64, 4),           \
    MODAP_SHAPE(256, 256, 2), MODAP_SHAPE(256, 256, 4), MODAP_SHAPE(256, 256, 8),        \
    MODAP_SHAPE(512, 512, 2), MODAP_SHAPE(512, 512, 4), MODAP_SHAPE(512, 512, 8),        \
    MODAP_SHAPE(1024, 1024, 2), MODAP_SHAPE(1024, 1024, 4)
#include "sweep_inst.inc"
