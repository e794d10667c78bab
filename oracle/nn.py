"""FP64 oracle of the gauge-covariant parallel-transport network used as a
flexible preconditioner, its losses and gradients, and flexible CG.

Test infrastructure only: see the package docstring. None of this is in the
paper; the layer form, losses and optimiser are project decisions.

Layer (channels C_in -> C_out) on the full 5D lattice, 20 terms per channel
pair, each a complex weight times a gauge-covariant operator:
    y_o = sum_i sum_t W[t, o, i] S_t X_i
    S_0 = P_+,  S_1 = P_-                                   (site local, chirality split)
    S_{2+mu} = T_{+mu},  S_{6+mu} = T_{-mu}                 (parallel transport)
    S_{10+mu} = gamma_mu T_{+mu},  S_{14+mu} = gamma_mu T_{-mu}
    S_18 psi(x, s) = P_+ psi(x, s-1),  S_19 psi(x, s) = P_- psi(x, s+1)   (cyclic in s)
    T_{+mu} psi(x) = U_mu(x) psi(x + mu),  T_{-mu} psi(x) = U_mu(x - mu)^dag psi(x - mu)
with the fermion boundary phases on hops across the lattice edge. With a
hop term in 1 and in gamma_mu each direction can weigh the two spin
projections (1 -+ gamma_mu) of the Wilson hop separately, and the s terms
the chirality-split coupling along the fifth dimension of D~ and M_ee.
Every S_t commutes with gauge transformations.

Network: B = L_n ... L_1 (channels 1 -> C -> ... -> 1) and N = B^dag B,
Hermitian and positive semi-definite by construction (<x, N x> = |B x|^2),
so flexible CG with N behaves like preconditioned CG. Its input is the
odd-sublattice residual embedded in the full lattice (even sites zero), its
output is read back on the odd sites.

Losses (project decisions):
* error loss over pairs (r, e):   sum_p |N(r_p)_odd - e_p|^2 / |e_p|^2;
* residual loss over vectors r:   sum_p min_c |c A N(r_p)_odd - r_p|^2 / |r_p|^2
      = sum_p [1 - |<A y_p, r_p>|^2 / (|A y_p|^2 |r_p|^2)],  y_p = N(r_p)_odd,
  for a Hermitian operator A on the odd sublattice (here A = M^dag M of the
  Schur system): the scale of N does not matter to CG, so it is left out.
Gradients are dL/dW* (Wirtinger); dL/dRe W = 2 Re(dL/dW*), dL/dIm W = 2 Im(dL/dW*).
"""
import numpy as np

from .lattice import GAMMA, P_PLUS, P_MINUS, shift, dagger, restrict, vdot, norm2

NTERMS = 20
S_AXIS = -7


def _colour(u, f):
    return np.einsum("...ab,...sb->...sa", u, f)


def _spin(m, f):
    return np.einsum("st,...tc->...sc", m, f)


def _hop(U, psi, mu, fwd, bc):
    if fwd:
        return _colour(U[mu], shift(psi, mu, +1, bc[mu]))
    return _colour(dagger(shift(U[mu], mu, -1)), shift(psi, mu, -1, bc[mu]))


def term(U, psi, t, bc, adj=False):
    """S_t psi, or S_t^dag psi (adj): T_{+mu}^dag = T_{-mu}, gamma_mu Hermitian and
    commuting with the transports, the s shifts reversed."""
    if t == 0:
        return _spin(P_PLUS, psi)
    if t == 1:
        return _spin(P_MINUS, psi)
    if t < 18:
        k = (t - 2) % 8
        mu, fwd = k % 4, k < 4
        h = _hop(U, psi, mu, fwd != adj, bc)
        return h if t < 10 else _spin(GAMMA[mu], h)
    if t == 18:
        return _spin(P_PLUS, np.roll(psi, -1 if adj else 1, axis=S_AXIS))
    return _spin(P_MINUS, np.roll(psi, 1 if adj else -1, axis=S_AXIS))


def terms(U, X, bc, adj=False):
    """[NTERMS, C, ...] all terms of every channel of X [C, ...]."""
    return np.stack([np.stack([term(U, X[c], t, bc, adj) for c in range(X.shape[0])]) for t in range(NTERMS)])


def layer(U, W, X, bc):
    """W [NTERMS, C_out, C_in] complex, X [C_in, Ls, T, Z, Y, X, 4, 3]."""
    return np.einsum("toi,ti...->o...", W, terms(U, X, bc))


def layer_adjoint(U, W, G, bc):
    """Adjoint of ``layer`` in X: sum_{t,o} conj(W[t, o, i]) S_t^dag G_o."""
    return np.einsum("toi,to...->i...", np.conj(W), terms(U, G, bc, adj=True))


def weight_grad(U, X, G, bc):
    """D[t, o, i] = sum_x <S_t X_i, G_o> (conjugate on the first slot)."""
    Z = terms(U, X, bc)
    G2 = G.reshape(G.shape[0], -1)
    Z2 = Z.reshape(Z.shape[0], Z.shape[1], -1)
    return np.einsum("on,tin->toi", G2, np.conj(Z2))


def forward(U, Ws, r_odd, dims, bc):
    """N(r) = B^dag B r on the odd sites and the activations: X[0..n] of B
    (X[0] the embedded residual) and Y[n..0] of B^dag (Y[n] = X[n])."""
    X = [r_odd[None]]
    for W in Ws:
        X.append(layer(U, W, X[-1], bc))
    Y = [X[-1]]
    for W in reversed(Ws):
        Y.append(layer_adjoint(U, W, Y[-1], bc))
    return restrict(Y[-1][0], dims, 1), (X, Y[::-1])


def _backprop(U, Ws, acts, g_out, grads, bc):
    """Accumulate dL/dW* into grads given dL/dN(r)* = g_out (odd field).
    Adjoint layer k (Y[k-1] = L_k^dag Y[k]): dL/dW_k* += weight_grad(G, Y[k])
    with G = dL/dY[k-1]*, and dL/dY[k]* = L_k G; then the layers of B as usual:
    dL/dW_k* += weight_grad(X[k-1], G), dL/dX[k-1]* = L_k^dag G."""
    X, Y = acts
    n = len(Ws)
    G = g_out[None]
    for k in range(1, n + 1):
        grads[k - 1] += weight_grad(U, G, Y[k], bc)
        G = layer(U, Ws[k - 1], G, bc)
    for k in range(n, 0, -1):
        grads[k - 1] += weight_grad(U, X[k - 1], G, bc)
        if k > 1:
            G = layer_adjoint(U, Ws[k - 1], G, bc)


def loss_and_grads(U, Ws, pairs, dims, bc):
    """Error loss sum |N(r_p) - e_p|^2 / |e_p|^2 and dL/dW* for every layer."""
    L = 0.0
    grads = [np.zeros_like(W) for W in Ws]
    for r, e in pairs:
        y, acts = forward(U, Ws, r, dims, bc)
        ne = norm2(e)
        d = y - e
        L += norm2(d) / ne
        _backprop(U, Ws, acts, restrict(d / ne, dims, 1), grads, bc)
    return L, grads


def residual_loss_and_grads(U, Ws, rs, A, dims, bc):
    """Residual loss sum_p [1 - |<A y, r>|^2 / (|A y|^2 |r|^2)], y = N(r_p) on
    the odd sites, A Hermitian: with a = A y, c = <a, r>,
    dL/da* = (|c|^2 a - conj(c) |a|^2 r) / (|a|^4 |r|^2), dL/dy* = A dL/da*."""
    L = 0.0
    grads = [np.zeros_like(W) for W in Ws]
    for r in rs:
        y, acts = forward(U, Ws, r, dims, bc)
        a = A(y)
        c = vdot(a, r)
        na, nr = norm2(a), norm2(r)
        L += 1.0 - abs(c) ** 2 / (na * nr)
        ga = (abs(c) ** 2 * a - np.conj(c) * na * r) / (na * na * nr)
        _backprop(U, Ws, acts, restrict(A(ga), dims, 1), grads, bc)
    return L, grads


def bf16_round(a):
    """Round real and imaginary parts to bfloat16 (nearest even), back as float64."""
    def r(x):
        b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
        b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
        return b.astype(np.uint32).view(np.float32).astype(np.float64)
    return r(a.real) + 1j * r(a.imag)


def fcg(op_normal, apply_prec, rhs, tol=1e-10, max_iter=10000):
    """Flexible CG with one-term truncation (Notay 2000) on A x = rhs,
    A Hermitian positive definite, from x = 0:
        z = N(r);  p = z - (<A p_old, z>/<p_old, A p_old>) p_old;  q = A p;
        alpha = <p, r>/<p, q>;  x += alpha p;  r -= alpha q."""
    x = np.zeros_like(rhs)
    r = rhs.copy()
    n0 = np.sqrt(norm2(rhs))
    p_old = q_old = None
    it = 0
    while np.sqrt(norm2(r)) > tol * n0 and it < max_iter:
        z = apply_prec(r)
        if p_old is None:
            p = z
        else:
            p = z - (vdot(q_old, z) / vdot(p_old, q_old)) * p_old
        q = op_normal(p)
        alpha = vdot(p, r) / vdot(p, q)
        x = x + alpha * p
        r = r - alpha * q
        p_old, q_old = p, q
        it += 1
    return x, it
