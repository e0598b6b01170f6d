// runtime.hip -- error reporting and version of the C ABI.
#include "common.hpp"

namespace pf {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string& msg) { g_last_error = msg; }

pf_status fail(pf_status st, const std::string& msg) {
    set_error(msg);
    return st;
}

}  // namespace pf

extern "C" {

const char* pf_last_error(void) { return pf::g_last_error.c_str(); }

int pf_version(void) { return 10000; }  // 1.0.0

}  // extern "C"
