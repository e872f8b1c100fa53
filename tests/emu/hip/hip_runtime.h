// Host-emulation stand-in for <hip/hip_runtime.h> (tests only).
#pragma once
#include "../hipemu.h"
