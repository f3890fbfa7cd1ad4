"""Lattices and the quasi-1D snake order (oracle; test infrastructure only).

Paper: main text, Hubbard-model paragraph (cylinders CL WxL periodic across
the width W and open along the length L; open squares OS with all edges
open), and Fig. 1a, whose thick path runs down one column of W sites,
crosses to the next column at the bottom, runs up it, crosses at the top,
and so on.

Reading used here: column x is traversed top-to-bottom (y = W-1 .. 0) when x
is even and bottom-to-top when x is odd.  The wrap bond (y=0, y=W-1) of a
cylinder is added only for W >= 3 (for W = 2 it would double the vertical
bond).  geometry: 0 = chain with open ends (W = 1), 1 = cylinder, 2 = open
square.
"""

CHAIN, CYLINDER, OPEN_SQUARE = 0, 1, 2


def snake_order(W, L):
    """List of (x, y) coordinates in chain order along the snake path."""
    order = []
    for x in range(L):
        ys = range(W - 1, -1, -1) if x % 2 == 0 else range(W)
        for y in ys:
            order.append((x, y))
    return order


def nn_bonds(W, L, geometry):
    """Nearest-neighbour bonds as sorted pairs (i, j), i < j, of chain indices."""
    if geometry == CHAIN and W != 1:
        raise ValueError("a chain has W = 1")
    order = snake_order(W, L)
    index = {xy: k for k, xy in enumerate(order)}
    edges = set()
    for (x, y) in order:
        # neighbour along the length (open ends)
        if x + 1 < L:
            edges.add(tuple(sorted((index[(x, y)], index[(x + 1, y)]))))
        # neighbour across the width
        if y + 1 < W:
            edges.add(tuple(sorted((index[(x, y)], index[(x, y + 1)]))))
        elif geometry == CYLINDER and W >= 3:
            edges.add(tuple(sorted((index[(x, y)], index[(x, 0)]))))
    return sorted(edges)


def pairs_at_distance(W, L, geometry, d2):
    """Pairs (i, j), i < j, of chain indices whose squared lattice distance is
    d2: dx^2 + dy^2 with dy taken the short way round a cylinder's width (W >=
    3), as in the spin correlation F(d) of the main text (average over the
    pairs at distance d)."""
    if geometry == CHAIN and W != 1:
        raise ValueError("a chain has W = 1")
    order = snake_order(W, L)
    out = []
    for i, (xi, yi) in enumerate(order):
        for j in range(i + 1, len(order)):
            xj, yj = order[j]
            dy = abs(yi - yj)
            if geometry == CYLINDER and W >= 3:
                dy = min(dy, W - dy)
            if (xi - xj) ** 2 + dy ** 2 == d2:
                out.append((i, j))
    return out


def nnn_bonds(W, L, geometry):
    """Next-nearest-neighbour pairs of SM Eq. S1: the diagonal neighbours
    (squared distance 2; a chain has none)."""
    return pairs_at_distance(W, L, geometry, 2)
