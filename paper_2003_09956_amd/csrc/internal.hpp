// Entry points shared between the translation units of the library that are
// not part of the C ABI.
#pragma once

#include <stdint.h>

#include "modap.h"

// The FP64 certificate of the stops of the given batch systems (each a no-op
// unless the system's committed state is an uncertified stop).  Synchronises.
modap_status modap_batch_certify_ids(modap_batch *batch, const modap_params *p, const int64_t *ids, int64_t count);
