// Host-side GP weight generation (quadruple precision), internal to the library.
#ifndef GPMOOD_GP_WEIGHTS_H
#define GPMOOD_GP_WEIGHTS_H

namespace gpm {

// Quarter-basis weights of one radius for both directions:
// w[dir][slot][k], dir 0 = x faces (face x+, nodes +g), dir 1 = y faces (face y+,
// nodes +g), k over the first kNQ[R] entries of kQ.  Values rounded from quad
// precision to double (w64) and, separately, to float (w32).
struct GpwLevel {
    int R;
    double w64[2][2][25];
    float w32[2][2][25];
    double qw64[2];  // Gauss weights of the stored slots (pair member / centre node)
    float qw32[2];
    double dlw64[2][2][25];  // d w / d log(ell) (the adjoint's ell gradient)
};

// u2 curvature weights (App. B, GP-R1 stencil, at the cell centre, unnormalised),
// per direction d: [0] centre cell, [1] the two neighbours along d, [2] the two
// neighbours across d.
struct GpwCurv {
    double w64[2][3];
    float w32[2][3];
};

// 3D weights of radius R (1 or 2) on the L1-ball stencil (kBall order): for each
// face f (x-, x+, y-, y+, z-, z+) and node k (q x q tensor nodes, q = R + 1, first
// tangential axis outer) the normalised prediction vector over the stencil, and
// the node weights.
struct Gpw3Level {
    int R;
    int nq;  // nodes per face
    double z64[6][9][25];
    float z32[6][9][25];
    double qw64[9];
    float qw32[9];
    // R = 2: the parity-basis weights of each face's four node classes (kPar3
    // entries; the orbit averages of the canonical node's prediction vector with
    // the component's signs), zero where a class does not use the component
    double pz64[6][4][25];
    float pz32[6][4][25];
};

// 3D u2 curvature weights per direction d on the R = 1 ball: [0] centre, [1] the
// two neighbours along d, [2] and [3] the two neighbours along each other axis
// (in x, y, z order).
struct Gpw3Curv {
    double w64[3][4];
    float w32[3][4];
};

// ax = ell/dx, ay = ell/dy.  Returns 0, or -1 if the covariance matrix is not
// numerically positive definite in quad precision.
// Stencil shapes of gpw_level: the blocky diamond, the cross (its cells on the
// axes), and POL-MOOD3 (radius 1, polynomial weights).
enum { GPW_DIAMOND = 0, GPW_CROSS = 1, GPW_POLY3 = 2 };
int gpw_level(int R, double ax, double ay, int shape, GpwLevel *out);
int gpw_curvature(double ax, double ay, double ell, GpwCurv *out);
int gpw3_level(int R, double ax, double ay, double az, Gpw3Level *out);
int gpw3_curvature(double ax, double ay, double az, double ell, Gpw3Curv *out);

}  // namespace gpm

#endif
