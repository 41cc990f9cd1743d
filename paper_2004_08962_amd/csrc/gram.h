#pragma once

#include "common.h"

namespace hicu {

size_t gram_workspace(const Geo& g);
int32_t launch_gram(const Geo& g, const void* x, void* G, void* ws, size_t ws_bytes, hipStream_t st);
// 1 = shift-correlation route (default, up to 32 coils), 0 = direct products.
int gram_route();
void set_gram_route(int route);

}  // namespace hicu
