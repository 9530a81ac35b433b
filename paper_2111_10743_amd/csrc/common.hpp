// Shared host-side helpers of the library: status codes, the thread-local
// error message and small dense linear algebra.
#pragma once
#include <cstdint>
#include <cstdio>
#include <cstdarg>
#include <string>
#include <vector>
#include <stdexcept>

#include "../../include/lb.h"

namespace lb {

// Thrown inside the library, turned into a status code at the C boundary.
struct Error : std::runtime_error {
  lb_status code;
  Error(lb_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] inline void fail(lb_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  throw Error(code, buf);
}

void set_last_error(const std::string& msg);

// In-place inverse of a dense row-major n x n matrix (Gauss-Jordan with
// partial pivoting).  Throws LB_EINVAL when singular.
void invert(std::vector<double>& A, int n);

}  // namespace lb
