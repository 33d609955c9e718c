// Host-side helpers shared by the entry points of libkftrack.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/libkftrack.h"

// Records the HIP error (if any) of the last launch; returns KF_OK or KF_E_HIP.
int kf_check_launch();
// Records a HIP error code from a runtime call; returns KF_OK or KF_E_HIP.
int kf_check(hipError_t e);
// Records a message for kf_last_error and returns status.
int kf_fail(int status, const char* msg);
int kf_check_geometry(const kf_geometry* g);
int kf_check_detector(const kf_detector* d);
