// Batched gradient steps over many problems (see batch.hip).
#pragma once

#include "common.h"
