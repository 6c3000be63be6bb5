// Driver for a sanitizer build (-fsanitize=address,undefined) of the device
// pair arithmetic compiled for the CPU (pair_math_host.cpp): blocks and pair
// gradients for far, overlapping, coincident and near-wall pairs in both
// precisions; the block must be the transpose of the block of the swapped
// pair (reciprocity) and every output finite.
#include <cmath>
#include <cstdio>

extern "C" {
void host_block_f64(const double* d, const double* z, double* out);
void host_block_f32(const double* d, const double* z, double* out);
void host_grad_f64(const double* d, const double* z, const double* v, double* out);
void host_grad_f32(const double* d, const double* z, const double* v, double* out);
}

int main() {
    int fails = 0;
    const double cases[][5] = {{3.0, -1.0, 0.5, 2.0, 1.5}, {0.3, 0.2, 0.1, 1.2, 1.1}, {0.0, 0.0, 0.0, 1.0, 1.0},
                               {1.9, 0.0, 0.0, 1.0, 1.0},  {40.0, 7.0, 2.0, 6.0, 4.0}};
    const double v[12] = {0.3, -0.2, 0.7, 0.5, 0.1, -0.6, -0.4, 0.9, 0.1, 0.2, -0.8, 0.4};
    for (const auto& c : cases) {
        const double d[3] = {c[0], c[1], c[2]}, z[2] = {c[3], c[4]};
        const double dm[3] = {-c[0], -c[1], -c[2]}, zm[2] = {c[4], c[3]};
        double b[9], bt[9], bf[9], gr[6], grf[6];
        host_block_f64(d, z, b);
        host_block_f64(dm, zm, bt);
        host_block_f32(d, z, bf);
        host_grad_f64(d, z, v, gr);
        host_grad_f32(d, z, v, grf);
        for (int r = 0; r < 3; ++r)
            for (int col = 0; col < 3; ++col)
                if (std::fabs(b[3 * r + col] - bt[3 * col + r]) > 1e-14 || !std::isfinite(bf[3 * r + col])) ++fails;
        for (int i = 0; i < 6; ++i)
            if (!std::isfinite(gr[i]) || !std::isfinite(grf[i])) ++fails;
    }
    std::printf(fails ? "sanitize-pair-math: %d failures\n" : "sanitize-pair-math: ok\n", fails);
    return fails ? 1 : 0;
}
