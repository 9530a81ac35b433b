// The kernels of the stored corrections, in this order (Section 3):
// S, dS/dx1, dS/dx2, dS/dx3, S', S''+D', D.
#pragma once

namespace lb {
constexpr int NKER = 7;
}  // namespace lb
