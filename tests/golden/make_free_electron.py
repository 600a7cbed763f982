"""Writes free_electron_chi0bar.txt: the closed-form chi0bar eigenvalues of the free-electron
model with one occupied plane wave, for the 10 bohr cubic cell at 5 Ha (16^3 grid).

chi0bar = v^(1/2) chi0 v^(1/2) on S' (Sec. 2.3, the symmetrised static response).  With V = 0
the orbitals are plane waves e^{iGr} / sqrt(Omega), eps_G = |G|^2 / 2.  With only G = 0
occupied, the sum over states that the Sternheimer solution reproduces (Sec. 2.3) couples
the occupied state to G alone: each excitation 0 -> G contributes
|<G|e^{iGr}|0>|^2 / (eps_0 - eps_G) = -2 / |G|^2, counted twice (the two terms of the static
response) and for two spins, so chi0(G, G) = -8 / (Omega |G|^2) and chi0 is diagonal in G.
With v(G) = 4 pi / |G|^2: lambda_G = v(G) chi0(G, G) = -32 pi / (Omega |G|^4).
Pure arithmetic: no oracle, no library.
"""
import math
import os

L = 10.0
ECUT = 5.0
OMEGA = L ** 3


def shells(nmax=4):
    out = {}
    for i in range(-nmax, nmax + 1):
        for j in range(-nmax, nmax + 1):
            for k in range(-nmax, nmax + 1):
                if (i, j, k) == (0, 0, 0):
                    continue
                g2 = (2 * math.pi / L) ** 2 * (i * i + j * j + k * k)
                if 0.5 * g2 > ECUT:
                    continue
                out[(i, j, k)] = -32 * math.pi / (OMEGA * g2 * g2)
    return out


def main():
    vals = shells()
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "free_electron_chi0bar.txt")
    with open(path, "w") as f:
        f.write("# Free-electron chi0bar eigenvalues, one occupied plane wave (G = 0), V = 0\n")
        f.write("# cell 10 bohr cube, E_cut 5 Ha, Hartree units, two spins\n")
        f.write("# closed form lambda_G = -32 pi / (Omega |G|^4) (Sec. 2.3 sum over states; derivation\n")
        f.write("# in make_free_electron.py).  Lowest |G| shells, one line per Miller index:\n")
        f.write("# m1 m2 m3 lambda\n")
        keys = sorted(vals, key=lambda t: (t[0] ** 2 + t[1] ** 2 + t[2] ** 2, t))
        for key in keys[:32]:
            f.write("%d %d %d %.17e\n" % (key[0], key[1], key[2], vals[key]))


if __name__ == "__main__":
    main()
