// Internal host-side declarations of libpm (not part of the C ABI).
#pragma once
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

namespace pm {

// One stored nonzero of M_d (eq. (3)); both (i, j) and (j, i) are present.
struct FluxEntry {
    int row, col, dir;
    double val;
};

inline int moment_index(int l, int m) { return l * l + l + m; }
void moment_lm(int i, int& l, int& m);

// Closed-form nonzeros of M_x, M_y, M_z for the orthonormal real harmonics.
std::vector<FluxEntry> flux_entries(int N);

// Parity bits ox | oy << 1 | oz << 2 of moment (l, m): the staggered grid.
int grid_bits(int l, int m);

// Position of a grid in the storage order G111, G221, G212, G122, G211,
// G121, G112, G222.
int grid_order(int bits);
extern const int kGridOfOrder[8];

struct Layout {
    int N = 0, V = 0;
    std::vector<int> slot_of;    // canonical moment -> storage slot
    std::vector<int> moment_of;  // storage slot -> canonical moment
    std::vector<int> order_of;   // canonical moment -> grid storage order 0..7
    int grid_begin[9] = {0};     // slots of grid g are [grid_begin[g], grid_begin[g+1])
};
Layout make_layout(int N);

// Largest Gauss-Legendre node of order N+1 = spectral radius of M_d.
double lambda_max(int N);

}  // namespace pm
