// Thread-local error message of the library (returned by dqmc_last_error), shared by its
// translation units.
#pragma once

#include <string>

#include "dqmc.h"

namespace dqmc {
dqmc_status set_error(dqmc_status s, const std::string& msg);
}
