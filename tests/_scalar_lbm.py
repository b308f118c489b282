"""Brute-force scalar restatement of one two-component step, for pinning the oracle.

Written independently of ``oracle/``: its own D3Q19 enumeration (velocities
found by scanning {-1,0,1}^3 for |c|^2 <= 2, weights by shell), explicit
modular neighbour indices, pull-form streaming instead of the oracle's push
form, and pure-Python loops over cells.  Only for grids of a few dozen cells.

Equations (arXiv 1601.01237, Sec. 2): (1) LBE, (2) BGK, (3) third-order
equilibrium with T0 = 1/3, (4)-(6) moments, (7) Shan-Chen force with the
pointwise wall potential of Sec. 4; forcing by the exact-difference reading.
"""

T0 = 1.0 / 3.0


def lattice():
    shell_weight = {0: 1.0 / 3.0, 1: 1.0 / 18.0, 2: 1.0 / 36.0}
    vel, w = [], []
    for cz in (-1, 0, 1):
        for cy in (-1, 0, 1):
            for cx in (-1, 0, 1):
                s = cx * cx + cy * cy + cz * cz
                if s <= 2:
                    vel.append((cx, cy, cz))
                    w.append(shell_weight[s])
    opp = [vel.index((-c[0], -c[1], -c[2])) for c in vel]
    return vel, w, opp


def feq(rho, u, c, w):
    cu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2]
    uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2]
    return rho * w * (1.0 + cu / T0 + cu * cu / (2 * T0 * T0) - uu / (2 * T0)
                      + cu ** 3 / (6 * T0 ** 3) - cu * uu / (2 * T0 * T0))


def step(f, shape, tau, G, solid, rho_wall, collision="bgk"):
    """One step.  ``f[s][q][(z, y, x)]`` nested lists/dicts in this module's order.

    ``solid`` is a set of (z, y, x) wall cells.  ``collision`` is "bgk"
    (Eq. 2), "regularized" (Eqs. 10-11 with the non-equilibrium part
    replaced by its second-order Hermite component) or "regularized3" (that
    plus its component along the contracted third-order polynomials, the
    energy flux).  Returns the new state.
    """
    vel, w, opp = lattice()
    nz, ny, nx = shape
    cells = [(z, y, x) for z in range(nz) for y in range(ny) for x in range(nx)]

    def nb(cell, c, sign=1):
        z, y, x = cell
        return ((z + sign * c[2]) % nz, (y + sign * c[1]) % ny, (x + sign * c[0]) % nx)

    rho = {}
    for cell in cells:
        if cell in solid:
            continue
        rho[cell] = [sum(f[s][q][cell] for q in range(19)) for s in range(2)]

    fstar = [[dict() for _ in range(19)] for _ in range(2)]
    for cell in cells:
        if cell in solid:
            continue
        ra, rb = rho[cell]
        rt = ra + rb
        j = [0.0, 0.0, 0.0]
        for s in range(2):
            for q in range(19):
                for a in range(3):
                    j[a] += vel[q][a] * f[s][q][cell]
        u = [j[a] / rt for a in range(3)]
        for s in range(2):
            # Eq. (7): force on species s from the other species.
            other = 1 - s
            acc = [0.0, 0.0, 0.0]
            for q in range(19):
                y = nb(cell, vel[q])
                rho_y = rho_wall[other] if y in solid else rho[y][other]
                for a in range(3):
                    acc[a] += w[q] * vel[q][a] * rho_y
            force = [G[s][other] * rho[cell][s] * acc[a] for a in range(3)]
            g = [force[a] / rho[cell][s] for a in range(3)]
            v = [u[a] + g[a] for a in range(3)]
            e_u = [feq(rho[cell][s], u, vel[q], w[q]) for q in range(19)]
            e_v = [feq(rho[cell][s], v, vel[q], w[q]) for q in range(19)]
            if collision in ("regularized", "regularized3"):
                # second moment of the non-equilibrium part, then its
                # Hermite-2 reconstruction w_q (c c - T0 I) : Pi / (2 T0^2)
                pi = [[sum(vel[q][a] * vel[q][b] * (f[s][q][cell] - e_u[q]) for q in range(19))
                       for b in range(3)] for a in range(3)]
                trace = pi[0][0] + pi[1][1] + pi[2][2]
                # energy flux: the contracted third-order polynomials
                # h_a(c) = sum_{b != a} (c_a c_b^2 - T0 c_a), their lattice
                # coefficients and their (lattice) norm
                energy = [0.0, 0.0, 0.0]
                hnorm = 0.0
                if collision == "regularized3":
                    def h(c, a):
                        return sum(c[a] * c[b] * c[b] - T0 * c[a] for b in range(3) if b != a)
                    energy = [sum(h(vel[q], a) * (f[s][q][cell] - e_u[q]) for q in range(19)) for a in range(3)]
                    hnorm = sum(w[q] * h(vel[q], 0) ** 2 for q in range(19))
            for q in range(19):
                fq = f[s][q][cell]
                if collision in ("regularized", "regularized3"):
                    cpc = sum(vel[q][a] * vel[q][b] * pi[a][b] for a in range(3) for b in range(3))
                    neq = w[q] * (cpc - T0 * trace) / (2.0 * T0 * T0)
                    if collision == "regularized3":
                        neq += w[q] * sum(h(vel[q], a) * energy[a] for a in range(3)) / hnorm
                    fstar[s][q][cell] = e_u[q] + (1.0 - 1.0 / tau[s]) * neq + (e_v[q] - e_u[q])
                else:
                    fstar[s][q][cell] = fq - (fq - e_u[q]) / tau[s] + (e_v[q] - e_u[q])

    new = [[dict() for _ in range(19)] for _ in range(2)]
    for cell in cells:
        for s in range(2):
            for q in range(19):
                if cell in solid:
                    new[s][q][cell] = 0.0
                    continue
                src = nb(cell, vel[q], sign=-1)
                if src in solid:
                    new[s][q][cell] = fstar[s][opp[q]][cell]
                else:
                    new[s][q][cell] = fstar[s][q][src]
    return new


def observables(f, shape, G, solid, rho_wall):
    """Per fluid cell (rho^A, rho^B, u_F) with u_F = u + (F^A + F^B) / (2 rho)
    (Eqs. 4-9): the mean of the mixture velocity before collision, j / rho,
    and after the force has added F^A + F^B.  Same state format as step()."""
    vel, w, _ = lattice()
    nz, ny, nx = shape
    out = {}
    rho = {}
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                cell = (z, y, x)
                if cell not in solid:
                    rho[cell] = [sum(f[s][q][cell] for q in range(19)) for s in range(2)]
    for cell, (ra, rb) in rho.items():
        z, y, x = cell
        j = [sum(vel[q][a] * (f[0][q][cell] + f[1][q][cell]) for q in range(19)) for a in range(3)]
        force = [0.0, 0.0, 0.0]
        for s in range(2):
            other = 1 - s
            for q in range(19):
                c = vel[q]
                y_ = ((z + c[2]) % nz, (y + c[1]) % ny, (x + c[0]) % nx)
                r = rho_wall[other] if y_ in solid else rho[y_][other]
                for a in range(3):
                    force[a] += G[s][other] * rho[cell][s] * w[q] * c[a] * r
        rt = ra + rb
        out[cell] = (ra, rb, [(j[a] + 0.5 * force[a]) / rt for a in range(3)])
    return out
