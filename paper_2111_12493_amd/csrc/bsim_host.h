// bsim_host.h -- host-only basics shared by the library and its CPU tests:
// the error the host code throws and a bit-width helper.
#pragma once

#include <cstdint>
#include <string>

namespace bsim {

// A failed call: status is a BSIM_E_* code, msg the text bsim_last_error
// returns.
struct DeviceError {
    int status;
    std::string msg;
};

// Bits needed to write x (0 for x = 0).
inline int bit_width(uint64_t x) {
    int b = 0;
    while (x) {
        b++;
        x >>= 1;
    }
    return b;
}

}  // namespace bsim
