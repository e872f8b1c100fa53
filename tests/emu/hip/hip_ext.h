// Emulation of <hip/hip_ext.h> for the host build (tests only).
#pragma once
#include "hip_runtime.h"
