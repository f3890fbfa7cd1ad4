"""Full-size check of the Hamiltonian MPO through the GPU path: at high
temperature the bilayer energy falls as E(beta_phys) = E_0 - beta_phys Var_0(H)
+ O(beta^2), and the infinite-temperature variance has a closed form:
Var_0(H) = N Var(U n_up n_dn - mu n) + t^2 N_bonds (every bond, both spins,
<(c+_i c_j + h.c.)^2>_0 = 1/2).  A missing or mis-weighted bond of the snake
MPO on a large lattice would show here."""
import pytest

from paper_2212_11973_amd import tantrg as T

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("W,L,geo,nbonds", [(10, 10, T.TT_OPEN_SQUARE, 180), (4, 16, T.TT_CYLINDER, 124),
                                            (6, 12, T.TT_CYLINDER, 138)])
def test_high_temperature_energy_slope(W, L, geo, nbonds):
    print("highT", W, L, flush=True)
    U, mu = 8.0, 2.0
    st = T.State.init(T.model(W, L, geo, 1.0, U, mu), T.options(D=400, symmetry=1, beta0=1e-5, seed=1))
    pts = []
    for db in (9e-5, 1e-4, 1e-4):
        st.sweep(db)
        o = st.observables()
        pts.append((o["beta_phys"], o["E"]))
    st.free()
    slope = (pts[2][1] - pts[0][1]) / (pts[2][0] - pts[0][0])
    var_loc = (2 * mu * mu + (U - 2 * mu) ** 2) / 4 - ((U - 4 * mu) / 4) ** 2
    var0 = W * L * var_loc + nbonds
    assert abs(slope + var0) <= 3e-3 * var0, (slope, var0)
