// Boundary-condition strings of the C interface (host only).
#pragma once

namespace vp {

// Transform code of a direction: periodic; walls at both ends (zero normal
// gradient, cosine transform DCT-II); outflow (p = 0 on the boundary face)
// at both ends (sine transform DST-II); a wall at the lower end and an
// outflow at the upper (quarter-wave cosine transform DCT-IV), or the
// reverse (the DCT-IV of the reversed line).
enum : int { BC_P = 0, BC_N = 1, BC_D = 2, BC_ND = 3, BC_DN = 4 };

// Per-end letters 'P', 'N' or 'D' of x-, x+, y-, y+, z-, z+ (upper case)
// from 3 letters (both ends of x, y, z alike) or 6 (one per end), either
// case.  VP_EINVAL for another length or letter, or a direction periodic at
// one end only.
int parse_ends(const char* bc, char ends[6]);

// Transform code of a direction whose ends are lo, hi (letters as above).
int direction_code(char lo, char hi);

// A length the x / y / spectral z transforms take: 2^k in [8, 1024],
// 3 * 2^k in [24, 768] or 5 * 2^k in [40, 640].
bool fft_length(int n);

}  // namespace vp
