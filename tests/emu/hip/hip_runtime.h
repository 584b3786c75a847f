// The kernel sources include <hip/hip_runtime.h>; in the host emulation that is the shim.
#pragma once
#include "../emu_hip.h"
