// bmg_weights.h -- the operator-induced interpolation weights of one fine
// vertex (section 2: collapse of the stencil onto a coarse line, from
// continuity of the normal flux; a cell centre eliminates its neighbours).
// The setup kernel that stores the weights and the pipelined finest pass that
// forms them from the rows it loads both call these expressions, so the two
// give the same bits.  Connections are positive (matrix entry = -connection).
#pragma once

namespace hbmg {

// Vertex on a coarse x-line: the stencil summed over each column,
//   den = C - N - S,  w_W = (W + NW + SW) / den,  w_E = (E + NE + SE) / den.
__device__ __forceinline__ void xline_weights(double c, double n, double s, double w, double nw, double sw,
                                              double e, double ne, double se, double &ww, double &we)
{
    const double den = c - n - s;
    const double aw = w + nw + sw;
    const double ae = e + ne + se;
    ww = aw / den;
    we = ae / den;
}

// Vertex on a coarse y-line: the stencil summed over each row,
//   den = C - E - W,  w_S = (S + SE + SW) / den,  w_N = (N + NE + NW) / den.
__device__ __forceinline__ void yline_weights(double c, double e, double w, double s, double se, double sw,
                                              double n, double ne, double nw, double &ws, double &wn)
{
    const double den = c - e - w;
    const double as = s + se + sw;
    const double an = n + ne + nw;
    ws = as / den;
    wn = an / den;
}

// Cell centre, weight on one coarse corner: the diagonal connection to that
// corner plus the two edge neighbours' line weights on it, over the diagonal.
__device__ __forceinline__ double centre_weight(double corner, double c1, double l1, double c2, double l2, double d)
{
    return (corner + c1 * l1 + c2 * l2) / d;
}

}  // namespace hbmg
