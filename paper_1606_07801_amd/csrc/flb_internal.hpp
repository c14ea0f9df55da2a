// Declarations shared by the translation units of the library.
#pragma once

#include <string>

#include "../../include/flb.h"
#include "flb_device.hpp"

namespace flb {

extern thread_local std::string g_err;
int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
double default_theta(int d);
int check_params(const flb_params* p);
template <typename T>
KParams<T> make_kparams(const flb_params& p, double rho_eq);

}  // namespace flb
