// Batched walk: placeholder translation unit until the persistent kernel lands.
#include "perm_device.hpp"
#include "perm_internal.hpp"
