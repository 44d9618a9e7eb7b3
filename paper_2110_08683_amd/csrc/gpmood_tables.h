// Internal tables shared by the host weight generator and the device kernels.
//
// The GP prediction vectors of a blocky-diamond stencil (Sec. "The GP stencil")
// have the mirror symmetries of the grid: the weights of face x- are those of
// face x+ mirrored in x, the weights of node -g are those of node +g mirrored
// along the face.  The library therefore stores each direction's weights for the
// + face and the positive nodes only, in a "quarter basis": for every quarter
// position (a, b) with a, b >= 0 and a + b <= R the four stencil values
// q(+-a, +-b) are combined into parity sums
//     EE = sum of all four, OE = odd in di, EO = odd in dj, OO = odd in both,
// and the weights into the matching combinations divided by the multiplicity.
// One set of products then yields the four states (+face/-face) x (+node/-node)
// by a two-stage butterfly (exact algebra, the identity
// sum_i w_i q_i = (1/4) (Hw)^T (Hq) with the 4x4 Hadamard matrix H).
//
// The entry list below is ordered so that radius 1 is a prefix of radius 2,
// which is a prefix of radius 3: the parity sums computed for the top order serve
// every lower order of the cascade.
#ifndef GPMOOD_TABLES_H
#define GPMOOD_TABLES_H

namespace gpm {

enum Comp { C_EE = 0, C_OE = 1, C_EO = 2, C_OO = 3 };

struct QEntry {
    int a, b, comp;
};

// Parity entries in order; radius R uses the first kNQ[R] of them.
constexpr QEntry kQ[25] = {
    {0, 0, C_EE},
    {1, 0, C_EE}, {1, 0, C_OE}, {0, 1, C_EE}, {0, 1, C_EO},
    {2, 0, C_EE}, {2, 0, C_OE}, {0, 2, C_EE}, {0, 2, C_EO},
    {1, 1, C_EE}, {1, 1, C_OE}, {1, 1, C_EO}, {1, 1, C_OO},
    {3, 0, C_EE}, {3, 0, C_OE}, {0, 3, C_EE}, {0, 3, C_EO},
    {2, 1, C_EE}, {2, 1, C_OE}, {2, 1, C_EO}, {2, 1, C_OO},
    {1, 2, C_EE}, {1, 2, C_OE}, {1, 2, C_EO}, {1, 2, C_OO},
};
constexpr int kNQ[4] = {1, 5, 13, 25};

// Gauss nodes per face for radius R (Step 3 of the stepwise algorithm: q = R + 1;
// FOG uses one node, its states are constant along the face).
constexpr int nodes_of(int R) { return R == 0 ? 1 : R + 1; }
// Distinct node slots stored per direction: one per +-g pair, plus the centre
// node of the 3-point rule (R = 2).
constexpr int slots_of(int R) { return R == 0 ? 0 : (R == 1 ? 1 : 2); }
// Is slot k the centre node (g = 0)?
constexpr bool slot_is_zero(int R, int k) { return R == 2 && k == 1; }

// Compact form for the cascade, which runs few faces per pass and is bound by
// latency and instruction fetch rather than arithmetic: the quarter positions
// (a, b) in the same order as kQ, radius R using the first kNP[R].  Each position
// is gathered as its four mirror cells (+-a, +-b); on an axis the mirror copies
// coincide, so its parity sums come out 2x (4x at the centre) and the table
// weights carry the matching factor 1/2 (1/4), which keeps every product exact.
constexpr int kNP[4] = {1, 3, 6, 10};
constexpr int kNPos = 10;
// a and b of position e, 4 bits each: (0,0) (1,0) (0,1) (2,0) (0,2) (1,1) (3,0) (0,3) (2,1) (1,2)
constexpr unsigned long long kPosA = 0x1203102010ull;
constexpr unsigned long long kPosB = 0x2130120100ull;
// Table layout [R 0..3][dir 0..1][slot 0..1][position 0..9][component 0..3],
// followed by the Gauss weights [R][slot] (R = 0: the single node, weight 1).
constexpr int kGtabPerDir = 2 * kNPos * 4;
constexpr int kGtabNodeOff = 4 * 2 * kGtabPerDir;
constexpr int kGtabSize = kGtabNodeOff + 4 * 2;

// 3D (GP-MOOD5 and lower): the stencil of radius R is the L1 ball |di|+|dj|+|dk|
// <= R, listed ring by ring so that radius 1 (7 cells) is a prefix of radius 2
// (25 cells).  A face carries q x q tensor Gauss nodes (q = R + 1), the first
// tangential axis (in x, y, z order) outer.
constexpr int kBall[25][3] = {
    {0, 0, 0},
    {-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1},
    {-2, 0, 0}, {2, 0, 0}, {0, -2, 0}, {0, 2, 0}, {0, 0, -2}, {0, 0, 2},
    {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 1, 0},
    {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1}, {1, 0, 1},
    {0, -1, -1}, {0, 1, -1}, {0, -1, 1}, {0, 1, 1},
};
constexpr int kNBall[3] = {1, 7, 25};

// Parity basis of the radius-2 ball seen from a face normal to axis A (normal
// offset dn, tangential offsets d1, d2 along the face's first and second
// tangential axes): the cells form orbits under d1 -> -d1 and d2 -> -d2, and entry
// e is the sum over the orbit of (dn, +-a1, +-a2) with the signs of component c
// (0: even-even, 1: odd in d1, 2: odd in d2, 3: odd in both).  A node at
// tangential signs (s1, s2) takes sum_e chi_c(s) W[e] P[e], with W the
// orbit-averaged weights of the class's canonical node: the 14 even entries come
// first, then the 5 odd-in-d1, the 5 odd-in-d2 and the one odd-odd entry.
struct Par3 {
    int dn, a1, a2, comp;
};
constexpr int kNPar3 = 25, kPar3EE = 14, kPar3OE = 5, kPar3EO = 5;
constexpr Par3 kPar3[kNPar3] = {
    {-2, 0, 0, 0}, {-1, 0, 0, 0}, {0, 0, 0, 0}, {1, 0, 0, 0}, {2, 0, 0, 0},
    {-1, 1, 0, 0}, {0, 1, 0, 0}, {1, 1, 0, 0}, {0, 2, 0, 0},
    {-1, 0, 1, 0}, {0, 0, 1, 0}, {1, 0, 1, 0}, {0, 0, 2, 0},
    {0, 1, 1, 0},
    {-1, 1, 0, 1}, {0, 1, 0, 1}, {1, 1, 0, 1}, {0, 2, 0, 1}, {0, 1, 1, 1},
    {-1, 0, 1, 2}, {0, 0, 1, 2}, {1, 0, 1, 2}, {0, 0, 2, 2}, {0, 1, 1, 2},
    {0, 1, 1, 3},
};
// Node classes of the 3 x 3 tensor nodes (node k = i1 * 3 + i2, i = 0, 1, 2 at
// tangential coordinate +g, 0, -g): 0 the centre (k = 4), 1 on the first
// tangential axis (k = 1, 7), 2 on the second (k = 3, 5), 3 the corners (k = 0,
// 2, 6, 8); canonical nodes 4, 1, 3, 0.
constexpr int kPar3Canon[4] = {4, 1, 3, 0};

// Ball index of the cell at offset (d[0], d[1], d[2]), -1 if outside the ball.
constexpr int ball_index(int dx, int dy, int dz)
{
    for (int m = 0; m < 25; ++m)
        if (kBall[m][0] == dx && kBall[m][1] == dy && kBall[m][2] == dz) return m;
    return -1;
}

}  // namespace gpm

#endif
