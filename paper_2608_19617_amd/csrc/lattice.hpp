// Velocity sets for the gfx950 kernels.
//
// D2Q9: the velocity matrix and weights of Sec. 2.1.1 in the printed order
// (rest, E, N, W, S, NE, NW, SW, SE), c_s^2 = 1/3. D3Q19: the textbook set
// used for the 3D scale-up (the paper is 2D); order rest, +x, -x, +y, -y,
// +z, -z, then the edges (+-x +-y), (+-x +-z), (+-y +-z), first sign
// slowest. Every loop over directions is unrolled so that c, w and the
// opposite table fold into immediates.
#pragma once

namespace lbm {

struct D2Q9 {
    static constexpr int Q = 9;
    static constexpr int D = 2;
    static constexpr int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    static constexpr int cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    static constexpr int cz[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    static constexpr int opp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
    static constexpr double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                                    1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
};

struct D3Q19 {
    static constexpr int Q = 19;
    static constexpr int D = 3;
    static constexpr int cx[19] = {0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1, 0, 0, 0, 0};
    static constexpr int cy[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1};
    static constexpr int cz[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1};
    static constexpr int opp[19] = {0, 2, 1, 4, 3, 6, 5, 10, 9, 8, 7, 14, 13, 12, 11, 18, 17, 16, 15};
    static constexpr double w[19] = {1.0 / 3,
                                     1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                                     1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                     1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
};

template <class L>
__host__ __device__ constexpr int comp(int a, int p) {
    return p == 0 ? L::cx[a] : (p == 1 ? L::cy[a] : L::cz[a]);
}

}  // namespace lbm
