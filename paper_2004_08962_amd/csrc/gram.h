#pragma once

#include "common.h"

namespace hicu {

size_t gram_workspace(const Geo& g);
int32_t launch_gram(const Geo& g, const void* x, void* G, void* ws, size_t ws_bytes, hipStream_t st);

}  // namespace hicu
