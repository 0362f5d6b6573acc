// Mode bits shared by host and device code of the codec library: the
// alphabet (standard or base64url, Section 2), strict decoding (Appendix A:
// leftover bits of the final quantum must be zero) and unpadded text.
#pragma once

constexpr int B64I_M_URL = 1;
constexpr int B64I_M_STRICT = 2;
constexpr int B64I_M_NOPAD = 4;
