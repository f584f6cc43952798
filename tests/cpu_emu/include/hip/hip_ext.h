// Host-only stand-in for <hip/hip_ext.h>: hipExtLaunchKernelGGL is
// provided by the stand-in hip_runtime.h of this folder.  TEST INFRASTRUCTURE.
#pragma once
#include "hip_runtime.h"
