"""Forward-error bounds for one iteration started from an identical state.

Two implementations that start an iteration from the same state differ only
by rounding: the summation order of the inner products and of nothing else
in the sparse products (rows are summed in storage order on both sides), and
the rounding of each vector statement (the GPU may fuse multiply-adds).

  * An inner product d = (u, v) formed in any order has |d_hat - d| <=
    n*u*sum|u_k v_k| (u = 2^-53), so two orders differ by at most
    2*n*u*sum|u_k v_k|.
  * Those errors go through each coefficient formula to first order.
  * Each vector statement v = sum_j c_j w_j then differs by at most
    sum_j (E(c_j)|w_j| + |c_j| E(w_j)) + 2*k_u*u*sum_j |c_j w_j|, where
    E(.) is the bound of an input (zero for loaded state) and k_u counts
    the roundings of the statement.
  * A product A w carries |A| E(w) + 2*L*u*|A||w| (L = longest row).

All magnitudes are taken from the oracle's own states at iterations k and
k+1; the returned bounds are used with a safety factor for the neglected
second-order terms.
"""
import numpy as np

U = np.finfo(np.float64).eps / 2


class Bounds:
    def __init__(self, A, st, st1):
        self.A = A
        self.M = A.to_scipy()
        self.absM = abs(self.M)
        self.n = A.n
        self.L = int(np.diff(A.rowptr).max()) if A.n else 0
        self.st, self.st1 = st, st1

    def dot(self, u, v):
        """value and absolute error bound of (u, v) between two summation orders"""
        return float(u @ v), 2.0 * self.n * U * float(np.abs(u) @ np.abs(v))

    def spmv(self, w, Ew):
        """bound of A w given an input bound Ew"""
        return self.absM @ Ew + 2.0 * self.L * U * (self.absM @ np.abs(w))

    @staticmethod
    def lin(terms, k_u=4):
        """bound of sum_j c_j w_j from (c, Ec, w, Ew) terms"""
        err = 0.0
        mag = 0.0
        for c, Ec, w, Ew in terms:
            err = err + Ec * np.abs(w) + abs(c) * Ew
            mag = mag + abs(c) * np.abs(w)
        return err + 2.0 * k_u * U * mag


def _ratio(num, Enum, den, Eden):
    """value and bound of num/den"""
    q = num / den
    return q, (Enum + abs(q) * Eden) / abs(den) + 2 * U * abs(q)


def safe_family(B: Bounds, variant: str, k: int, replace: bool):
    """Bounds on the state after iteration k of ssBiCGSafe2 / p-BiCGSafe(-rr)."""
    st, st1 = B.st, B.st1
    V = st.vec
    s, y, r, rs, t = V("s"), V("y"), V("r"), V("rs"), V("t")
    if variant == "ssbicgsafe2":
        s = B.M @ r  # formed at the top of the iteration from r_k (identical on both sides)
    a, Ea = B.dot(s, s)
    bb, Eb = B.dot(y, y)
    c, Ec = B.dot(s, y)
    d, Ed = B.dot(s, r)
    e, Ee = B.dot(y, r)
    f, Ef = B.dot(rs, r)
    g, Eg = B.dot(rs, s)
    h, Eh = B.dot(rs, t)
    if k == 0:
        beta, Ebeta = 0.0, 0.0
        alpha, Ealpha = _ratio(f, Ef, g, Eg)
        zeta, Ezeta = _ratio(d, Ed, a, Ea)
        eta, Eeta = 0.0, 0.0
    else:
        den_b = st.scal("zeta") * st.scal("f")
        beta, Ebeta = _ratio(st.scal("alpha") * f, abs(st.scal("alpha")) * Ef, den_b, 0.0)
        den_a = g + beta * h
        Eden_a = Eg + Ebeta * abs(h) + abs(beta) * Eh
        alpha, Ealpha = _ratio(f, Ef, den_a, Eden_a)
        den = a * bb - c * c
        Eden = Ea * abs(bb) + abs(a) * Eb + 2 * abs(c) * Ec
        zeta, Ezeta = _ratio(bb * d - c * e, Eb * abs(d) + abs(bb) * Ed + Ec * abs(e) + abs(c) * Ee,
                             den, Eden)
        eta, Eeta = _ratio(a * e - c * d, Ea * abs(e) + abs(a) * Ee + Ec * abs(d) + abs(c) * Ed,
                           den, Eden)
    coef = {"alpha": (alpha, Ealpha), "beta": (beta, Ebeta), "zeta": (zeta, Ezeta),
            "eta": (eta, Eeta), "f": (f, Ef)}
    z0 = np.zeros(B.n)
    p, u, zz, x, l, gg, w = V("p"), V("u"), V("z"), V("x"), V("l"), V("g"), V("w")
    E = {}
    Ep = B.lin([(1, 0, r, z0), (beta, Ebeta, p, z0), (-beta, Ebeta, u, z0)])
    o = s + beta * t
    Eo = B.lin([(1, 0, s, z0), (beta, Ebeta, t, z0)])
    yu = y + beta * u
    Eyu = B.lin([(1, 0, y, z0), (beta, Ebeta, u, z0)])
    un = zeta * o + eta * yu
    Eu = B.lin([(zeta, Ezeta, o, Eo), (eta, Eeta, yu, Eyu)])
    if variant == "ssbicgsafe2":
        wn = B.M @ un
        Ew = B.spmv(un, Eu)
        qn, Eq = None, None
    elif replace:
        qn = B.M @ o
        Eq = B.spmv(o, Eo)
        wn = B.M @ un
        Ew = B.spmv(un, Eu)
    else:
        As = B.M @ s
        qn = As + beta * l
        Eq = B.lin([(1, 0, As, z0), (beta, Ebeta, l, z0)])
        gw = gg + beta * w
        Egw = B.lin([(1, 0, gg, z0), (beta, Ebeta, w, z0)])
        wn = zeta * qn + eta * gw
        Ew = B.lin([(zeta, Ezeta, qn, Eq), (eta, Eeta, gw, Egw)])
    pn = r + beta * (p - u)
    Et = B.lin([(1, 0, o, Eo), (-1, 0, wn, Ew)])
    Ez = B.lin([(zeta, Ezeta, r, z0), (eta, Eeta, zz, z0), (-alpha, Ealpha, un, Eu)])
    zn = zeta * r + eta * zz - alpha * un
    yn = zeta * s + eta * y - alpha * wn
    Ey = B.lin([(zeta, Ezeta, s, z0), (eta, Eeta, y, z0), (-alpha, Ealpha, wn, Ew)])
    Ex = B.lin([(1, 0, x, z0), (alpha, Ealpha, pn, Ep), (1, 0, zn, Ez)])
    E.update(p=Ep, u=Eu, t=Et, z=Ez, y=Ey, x=Ex)
    if variant != "ssbicgsafe2":
        E["q"] = Eq
        E["w"] = Ew
    if replace:
        xn = x + alpha * pn + zn
        rn = B.A.b - B.M @ xn
        Er = np.abs(B.A.b) * 0 + B.spmv(xn, Ex) + 2 * U * (np.abs(B.A.b) + B.absM @ np.abs(xn))
        tn = o - wn
        E["r"] = Er
        E["l"] = B.spmv(tn, Et)
        E["g"] = B.spmv(yn, Ey)
        E["s"] = B.spmv(rn, Er)
    else:
        rn = r - alpha * o - yn
        Er = B.lin([(1, 0, r, z0), (-alpha, Ealpha, o, Eo), (-1, 0, yn, Ey)])
        E["r"] = Er
        if variant == "ssbicgsafe2":
            E["s"] = B.spmv(rn, Er)  # s_{k+1} = A r_{k+1}, formed when iteration k+1 starts
        else:
            Aw = B.M @ wn
            EAw = B.spmv(wn, Ew)
            As = B.M @ s
            E["l"] = B.lin([(1, 0, qn, Eq), (-1, 0, Aw, EAw)])
            gn = zeta * As + eta * gg - alpha * Aw
            Eg_ = B.lin([(zeta, Ezeta, As, z0), (eta, Eeta, gg, z0), (-alpha, Ealpha, Aw, EAw)])
            E["g"] = Eg_
            E["s"] = B.lin([(1, 0, s, z0), (-alpha, Ealpha, qn, Eq), (-1, 0, gn, Eg_)])
    return coef, E


def pbicgstab(B: Bounds, k: int):
    """Bounds on the state after iteration k of pipelined BiCGStab."""
    st, st1 = B.st, B.st1
    V, V1 = st.vec, st1.vec
    z0 = np.zeros(B.n)
    al, be, omp = st.scal("alpha"), st.scal("beta"), st.scal("omega")
    r, p, s, w, zz, t, v, x, rs = V("r"), V("p"), V("s"), V("w"), V("z"), V("t"), V("v"), V("x"), V("rs")
    E = {}
    E["p"] = B.lin([(1, 0, r, z0), (be, 0, p, z0), (-be * omp, 0, s, z0)], k_u=5)
    E["s"] = B.lin([(1, 0, w, z0), (be, 0, s, z0), (-be * omp, 0, zz, z0)], k_u=5)
    E["z"] = B.lin([(1, 0, t, z0), (be, 0, zz, z0), (-be * omp, 0, v, z0)], k_u=5)
    sn, zn = V1("s"), V1("z")
    E["q"] = B.lin([(1, 0, r, z0), (-al, 0, sn, E["s"])])
    E["y"] = B.lin([(1, 0, w, z0), (-al, 0, zn, E["z"])])
    q, y = V1("q"), V1("y")
    qy, Eqy = B.dot(q, y)
    yy, Eyy = B.dot(y, y)
    Eqy += 2 * abs(y) @ E["q"] + 2 * abs(q) @ E["y"]
    Eyy += 4 * abs(y) @ E["y"]
    om, Eom = (0.0, 0.0) if yy == 0 else _ratio(qy, Eqy, yy, Eyy)
    vn = B.M @ zn
    E["v"] = B.spmv(zn, E["z"])
    pn = V1("p")
    E["x"] = B.lin([(1, 0, x, z0), (al, 0, pn, E["p"]), (om, Eom, q, E["q"])])
    E["r"] = B.lin([(1, 0, q, E["q"]), (-om, Eom, y, E["y"])])
    tav = t - al * vn
    Etav = B.lin([(1, 0, t, z0), (-al, 0, vn, E["v"])])
    E["w"] = B.lin([(1, 0, y, E["y"]), (-om, Eom, tav, Etav)])
    rn, wn = V1("r"), V1("w")
    E["t"] = B.spmv(wn, E["w"])
    f, Ef = B.dot(rs, rn)
    gw, Egw = B.dot(rs, wn)
    gs, Egs = B.dot(rs, sn)
    gz, Egz = B.dot(rs, zn)
    rho, Erho = B.dot(rn, rn)
    Ef += abs(rs) @ E["r"]
    Egw += abs(rs) @ E["w"]
    Egs += abs(rs) @ E["s"]
    Egz += abs(rs) @ E["z"]
    Erho += 2 * abs(rn) @ E["r"]
    beta, Ebeta = _ratio(al * f, abs(al) * Ef, om * st.scal("f"), Eom * abs(st.scal("f")))
    den = gw + beta * gs - beta * om * gz
    Eden = Egw + Ebeta * abs(gs) + abs(beta) * Egs + (Ebeta * abs(om) + abs(beta) * Eom) * abs(gz) \
        + abs(beta * om) * Egz
    alpha, Ealpha = _ratio(f, Ef, den, Eden)
    coef = {"alpha": (alpha, Ealpha), "beta": (beta, Ebeta), "omega": (om, Eom), "f": (f, Ef),
            "rho": (rho, Erho), "gs": (gs, Egs), "gw": (gw, Egw), "gz": (gz, Egz)}
    return coef, E
