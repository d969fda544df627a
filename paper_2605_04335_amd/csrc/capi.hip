// Thread-local error message of the C ABI.
#include "common.hpp"

namespace ibm {
namespace {
thread_local std::string g_last_error;
}
void set_last_error(const std::string &msg) { g_last_error = msg; }
}  // namespace ibm

extern "C" const char *ibm_last_error(void) { return ibm::g_last_error.c_str(); }
