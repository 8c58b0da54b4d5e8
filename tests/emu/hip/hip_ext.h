// Launch with timing events (CPU emulation: the events are not recorded).
#pragma once
#include "hip_runtime.h"
#define hipExtLaunchKernelGGL(k, g, b, sh, st, e0, e1, fl, ...) emu_launch(k, dim3(g), dim3(b), __VA_ARGS__)
