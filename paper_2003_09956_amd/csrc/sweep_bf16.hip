// Fused sweep shapes for bfloat16 storage (16-byte vector = 8 elements).
#define MODAP_DT 2
#define MODAP_SHAPES                                                                     \
    MODAP_SHAPE(256, 64, 1), MODAP_SHAPE(256, 64, 2), MODAP_SHAPE(256, 64, 4),           \
    MODAP_SHAPE(256, 256, 2), MODAP_SHAPE(256, 256, 4),                                  \
    MODAP_SHAPE(512, 512, 2), MODAP_SHAPE(512, 512, 4),                                  \
    MODAP_SHAPE(1024, 1024, 2), MODAP_SHAPE(1024, 1024, 4)
#include "sweep_inst.inc"
