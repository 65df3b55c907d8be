#pragma once
#include <cstddef>
#include <cstdint>
#include <string>

namespace ffv {
// Lower-case hex SHA-256 digest of n bytes.
std::string sha256_hex(const uint8_t* data, size_t n);
}  // namespace ffv
