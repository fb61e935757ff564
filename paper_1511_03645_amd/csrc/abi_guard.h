// No C++ exception crosses the C ABI: the body of every entry point that can
// allocate on the host runs between WP_ABI_TRY and WP_ABI_CATCH, which turn
// an exception into a status code and a last-error message.  Host code only.
#pragma once

#include <exception>
#include <new>
#include <stdexcept>
#include <string>

#include "wp.h"

namespace wp {

// Inside a catch block: the status for the exception being handled
// (std::bad_alloc and std::length_error: a host allocation failed, WP_ENOMEM;
// anything else: the call could not complete, WP_ESTATE), with its message
// in *err when err is given.  Never throws.
inline int abi_exception_status(std::string *err) noexcept
{
    int code = WP_ESTATE;
    const char *what = "internal error";
    try {
        throw;
    } catch (const std::bad_alloc &) {
        code = WP_ENOMEM;
        what = "host allocation failed";
    } catch (const std::length_error &) {
        code = WP_ENOMEM;
        what = "host allocation too large";
    } catch (...) {
    }
    if (err) {
        try {
            *err = what;
        } catch (...) {
        }
    }
    return code;
}

}  // namespace wp

#define WP_ABI_TRY try {
#define WP_ABI_CATCH(err) \
    }                     \
    catch (...) { return ::wp::abi_exception_status(err); }
