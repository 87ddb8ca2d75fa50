// Test-only stand-in (see hip_runtime_api.h).
#pragma once
#include "hip_runtime_api.h"
