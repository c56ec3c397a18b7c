// Error-code boundary shared by every exported entry point (no HIP types, so
// the plain C++ planner includes it too).
#pragma once

#include <exception>
#include <new>
#include <string>

#include "sv.h"

namespace sv {

void set_error(const std::string &msg);
void clear_error();

// Every exported entry point runs its body through guard(): an exception
// thrown inside (a failed host allocation, an internal error) becomes an
// error code and a message, so none crosses the C interface.
template <typename F>
int guard(F &&f) noexcept {
  try {
    return f();
  } catch (const std::bad_alloc &) {
    set_error("host allocation failed");
    return SV_ERR_DEVICE;
  } catch (const std::exception &e) {
    set_error(std::string("internal error: ") + e.what());
    return SV_ERR_STATE;
  } catch (...) {
    set_error("internal error");
    return SV_ERR_STATE;
  }
}

}  // namespace sv
