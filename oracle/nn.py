"""FP64 oracle of the gauge-covariant parallel-transport network used as a
flexible preconditioner, its loss and gradients, and flexible CG.

Test infrastructure only: see the package docstring. None of this is in the
paper; the layer form, loss and optimiser are project decisions.

Layer (channels C_in -> C_out), on every s-slice of the full lattice:
    y_c(x) = sum_{c'} [ W[0, c, c'] X_{c'}(x)
                        + sum_mu W[1+mu, c, c'] T_{+mu} X_{c'}(x)
                        + sum_mu W[5+mu, c, c'] T_{-mu} X_{c'}(x) ]
    T_{+mu} psi(x) = U_mu(x) psi(x + mu),   T_{-mu} psi(x) = U_mu(x - mu)^dag psi(x - mu)
with the fermion boundary phases on hops across the lattice edge. The
weights are complex scalars: spin is untouched, colour is parallel
transported, so the layer is gauge covariant. The network is a stack of
layers; its input is the odd-sublattice residual embedded in the full lattice
(even sites zero) and its output is read back on the odd sites.

Losses (project decisions):
* error loss over pairs (r, e):   sum_p |N(r_p)_odd - e_p|^2 / |e_p|^2;
* residual loss over vectors r:   sum_p |A N(r_p)_odd - r_p|^2 / |r_p|^2 for a
  Hermitian operator A on the odd sublattice (here A = M^dag M of the Schur
  system), so that A N approximates the identity.
Gradients are dL/dW* (Wirtinger); dL/dRe W = 2 Re(dL/dW*), dL/dIm W = 2 Im(dL/dW*).
"""
import numpy as np

from .lattice import shift, dagger, restrict, vdot, norm2


def _colour(u, f):
    return np.einsum("...ab,...sb->...sa", u, f)


def transport(U, psi, t, bc):
    """Stencil term t: 0 identity, 1..4 forward mu = t-1, 5..8 backward mu = t-5."""
    if t == 0:
        return psi
    if t <= 4:
        mu = t - 1
        return _colour(U[mu], shift(psi, mu, +1, bc[mu]))
    mu = t - 5
    return _colour(dagger(shift(U[mu], mu, -1)), shift(psi, mu, -1, bc[mu]))


def transports(U, X, bc):
    """[9, C, ...] all stencil terms of every channel of X [C, ...]."""
    return np.stack([np.stack([transport(U, X[c], t, bc) for c in range(X.shape[0])]) for t in range(9)])


def layer(U, W, X, bc):
    """W [9, C_out, C_in] complex, X [C_in, Ls, T, Z, Y, X, 4, 3]."""
    Z = transports(U, X, bc)
    return np.einsum("toi,ti...->o...", W, Z)


def layer_adjoint(U, W, G, bc):
    """Adjoint of ``layer`` in X: sum_{t,c} conj(W[t,c,c']) T_t^dag G_c with T_{+mu}^dag = T_{-mu}."""
    swap = [0, 5, 6, 7, 8, 1, 2, 3, 4]
    out = np.zeros((W.shape[2],) + G.shape[1:], dtype=np.complex128)
    for t in range(9):
        TG = np.stack([transport(U, G[c], swap[t], bc) for c in range(G.shape[0])])
        out += np.einsum("oi,o...->i...", np.conj(W[t]), TG)
    return out


def weight_grad(U, X, G, bc):
    """dL/dW*[t, c, c'] = sum_x <T_t X_{c'}, G_c> with G = dL/dy*."""
    Z = transports(U, X, bc)
    G2 = G.reshape(G.shape[0], -1)
    Z2 = Z.reshape(Z.shape[0], Z.shape[1], -1)
    return np.einsum("on,tin->toi", G2, np.conj(Z2))


def forward(U, Ws, r_odd, dims, bc):
    """Network output on the odd sites and the activations [X0..X_L]."""
    X = [r_odd[None]]  # the embedded odd residual (even sites already zero)
    for W in Ws:
        X.append(layer(U, W, X[-1], bc))
    return restrict(X[-1][0], dims, 1), X


def loss_and_grads(U, Ws, pairs, dims, bc):
    """L = sum_p |N(r_p) - e_p|^2 / |e_p|^2 and dL/dW* for every layer."""
    L = 0.0
    grads = [np.zeros_like(W) for W in Ws]
    for r, e in pairs:
        y, X = forward(U, Ws, r, dims, bc)
        ne = norm2(e)
        d = y - e
        L += norm2(d) / ne
        G = (d / ne)[None]
        for k in range(len(Ws) - 1, -1, -1):
            grads[k] += weight_grad(U, X[k], G, bc)
            if k > 0:
                G = layer_adjoint(U, Ws[k], G, bc)
    return L, grads


def _backprop(U, Ws, X, G, grads, bc):
    for k in range(len(Ws) - 1, -1, -1):
        grads[k] += weight_grad(U, X[k], G, bc)
        if k > 0:
            G = layer_adjoint(U, Ws[k], G, bc)


def residual_loss_and_grads(U, Ws, rs, A, dims, bc):
    """L = sum_p |A y_p - r_p|^2 / |r_p|^2 with y_p = N(r_p) on the odd sites, A
    Hermitian; dL/dy* = A (A y - r) / |r|^2, then the same back-propagation."""
    L = 0.0
    grads = [np.zeros_like(W) for W in Ws]
    for r in rs:
        y, X = forward(U, Ws, r, dims, bc)
        nr = norm2(r)
        d = A(y) - r
        L += norm2(d) / nr
        _backprop(U, Ws, X, (A(d) / nr)[None], grads, bc)
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
