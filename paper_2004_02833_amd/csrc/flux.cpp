// Host setup: flux matrices, staggered-grid assignment, storage layout.
//
// Flux matrices (paper Sec. 2, eq. (3)).  The paper does not print the
// entries of the symmetric sparse M_x, M_y, M_z.  For orthonormal real
// spherical harmonics R_{l,m} (z polar axis, cos(m phi) for m > 0,
// sin(|m| phi) for m < 0, no Condon-Shortley sign) they follow from the
// standard recurrences for mu Y_l^m and sqrt(1-mu^2) e^{+-i phi} Y_l^m.
// Each couples degree l with l+1 only:
//   M_z: (l, m) -- (l+1, m)             a(l,|m|) = sqrt(((l+1)^2 - m^2) / ((2l+1)(2l+3)))
//   M_x: |m| -> |m|+1 keeps the cos/sin type, value b+(l,|m|) (sqrt 2 at m = 0);
//        |m| -> |m|-1 keeps the type, value -b-(l,|m|) (sqrt 2 at |m| = 1)
//   M_y: the same couplings with the cos/sin type swapped and signs as below
//   b+-(l,mu) = 1/2 sqrt((l+-mu+1)(l+-mu+2) / ((2l+1)(2l+3))).
// The result has 1..4 nonzeros per row in M_x and M_y and 0..2 in M_z
// (Sec. 3.2, "Unroll multiplications").
//
// Grid assignment (Sec. 2.1): moment i sits on G_{1+ox,1+oy,1+oz} where o_d
// is 1 iff R_i is odd under Omega_d -> -Omega_d.  For R_{l,m}:
//   m >= 0: (ox, oy, oz) = (m mod 2, 0, (l+m) mod 2)
//   m <  0: (ox, oy, oz) = ((|m|+1) mod 2, 1, (l+|m|) mod 2)
// so a d-derivative always joins grids that differ exactly in index d, and
// ox + oy + oz = l (mod 2): even grids hold even l, odd grids odd l.
#include <cmath>

#include "pm_internal.h"

namespace pm {

const int kGridOfOrder[8] = {0, 3, 5, 6, 1, 2, 4, 7};  // G111 G221 G212 G122 G211 G121 G112 G222

void moment_lm(int i, int& l, int& m) {
    l = (int)std::floor(std::sqrt((double)i));
    while ((l + 1) * (l + 1) <= i) ++l;
    while (l * l > i) --l;
    m = i - l * l - l;
}

int grid_bits(int l, int m) {
    int mu = m < 0 ? -m : m;
    int ox, oy, oz;
    if (m >= 0) {
        ox = mu & 1;
        oy = 0;
    } else {
        ox = (mu + 1) & 1;
        oy = 1;
    }
    oz = (l + mu) & 1;
    return ox | (oy << 1) | (oz << 2);
}

int grid_order(int bits) {
    for (int g = 0; g < 8; ++g)
        if (kGridOfOrder[g] == bits) return g;
    return -1;
}

std::vector<FluxEntry> flux_entries(int N) {
    std::vector<FluxEntry> e;
    auto put = [&](int d, int a, int b, double v) {
        e.push_back({a, b, d, v});
        e.push_back({b, a, d, v});
    };
    const double s2 = std::sqrt(2.0);
    for (int l = 0; l < N; ++l) {
        const double den = (double)(2 * l + 1) * (double)(2 * l + 3);
        for (int m = -l; m <= l; ++m) {
            const int mu = m < 0 ? -m : m;
            put(2, moment_index(l, m), moment_index(l + 1, m),
                std::sqrt(((double)(l + 1) * (l + 1) - (double)mu * mu) / den));
            // |m| -> |m| + 1
            double c = 0.5 * std::sqrt((double)(l + mu + 1) * (double)(l + mu + 2) / den);
            if (mu == 0) c *= s2;
            if (m >= 0) {
                put(0, moment_index(l, mu), moment_index(l + 1, mu + 1), c);
                put(1, moment_index(l, mu), moment_index(l + 1, -(mu + 1)), c);
            } else {
                put(0, moment_index(l, -mu), moment_index(l + 1, -(mu + 1)), c);
                put(1, moment_index(l, -mu), moment_index(l + 1, mu + 1), -c);
            }
            // |m| -> |m| - 1
            if (mu >= 1) {
                double cm = 0.5 * std::sqrt((double)(l - mu + 1) * (double)(l - mu + 2) / den);
                if (mu == 1) cm *= s2;
                if (m > 0) {
                    put(0, moment_index(l, mu), moment_index(l + 1, mu - 1), -cm);
                    if (mu >= 2) put(1, moment_index(l, mu), moment_index(l + 1, -(mu - 1)), cm);
                } else {
                    if (mu >= 2) put(0, moment_index(l, -mu), moment_index(l + 1, -(mu - 1)), -cm);
                    put(1, moment_index(l, -mu), moment_index(l + 1, mu - 1), -cm);
                }
            }
        }
    }
    return e;
}

Layout make_layout(int N) {
    Layout L;
    L.N = N;
    L.V = (N + 1) * (N + 1);
    L.slot_of.assign(L.V, -1);
    L.order_of.assign(L.V, -1);
    for (int i = 0; i < L.V; ++i) {
        int l, m;
        moment_lm(i, l, m);
        L.order_of[i] = grid_order(grid_bits(l, m));
    }
    int s = 0;
    for (int g = 0; g < 8; ++g) {
        L.grid_begin[g] = s;
        for (int i = 0; i < L.V; ++i)
            if (L.order_of[i] == g) {
                L.slot_of[i] = s++;
                L.moment_of.push_back(i);
            }
    }
    L.grid_begin[8] = s;
    return L;
}

double lambda_max(int N) {
    // Largest root of P_{N+1} by Newton from the Chebyshev-type guess.
    const int n = N + 1;
    if (n == 1) return 0.0;
    double x = std::cos(M_PI * (1.0 - 0.25) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
        double p0 = 1.0, p1 = x;
        for (int k = 2; k <= n; ++k) {
            double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        double dp = n * (x * p1 - p0) / (x * x - 1.0);
        double dx = p1 / dp;
        x -= dx;
        if (std::fabs(dx) < 1e-16) break;
    }
    return x;
}

}  // namespace pm
