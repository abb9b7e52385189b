// Boundary-condition strings of the C interface (host only).
#pragma once

namespace vp {

// Transform code of a direction: periodic; walls at both ends (zero normal
// gradient, cosine transform); outflow (p = 0 on the boundary face) at both
// ends (sine transform).  The z pass also takes a wall at one end and an
// outflow at the other (zsolve).
enum : int { BC_P = 0, BC_N = 1, BC_D = 2 };

// Per-end letters 'P', 'N' or 'D' of x-, x+, y-, y+, z-, z+ (upper case)
// from 3 letters (both ends of x, y, z alike) or 6 (one per end), either
// case.  VP_EINVAL for another length or letter, or a direction periodic at
// one end only.
int parse_ends(const char* bc, char ends[6]);

// Transform code (BC_P, BC_N or BC_D) of a direction whose ends are lo, hi;
// -1 for a wall at one end and an outflow at the other (no x / y transform).
int direction_code(char lo, char hi);

}  // namespace vp
