"""Python binding of libgocp: argument marshalling only.

Every function forwards to the C ABI entry point of the same name (see
include/gocp.h); all computation happens in the library.  Device buffers are
torch tensors on a ROCm device (complex128 or complex64, contiguous); torch
supplies memory and streams, nothing else.
"""

from __future__ import annotations

import ctypes as C

import numpy as np

from ._lib import load, check, AdaptParams, AdaptResult, ReoptParams, ReoptResult, RequestInfo, GOCP_EBUSY

__all__ = ["MAPPINGS", "Hamiltonian", "Pool", "Context", "pauli_hamiltonian_load",
           "pauli_hamiltonian_load_terms", "pool_build", "pool_build_pauli", "taylor5_apply_family", "gocp_partition", "hf_index",
           "basis_occupation", "state_hf", "sector_weight",
           "state_basis", "energy", "apply_hamiltonian", "pool_gradients", "pool_gradients_noalloc",
           "taylor5_apply",
           "adapt_solve", "adapt_reopt_solve", "Batch", "Server", "request_footprint", "version",
           "phase_trace"]

MAPPINGS = {"jw": 0, "bk": 1, 0: 0, 1: 1}
C128, C64 = 0, 1


def _mapping(m) -> int:
    if m not in MAPPINGS:
        raise ValueError(f"mapping must be 'jw' or 'bk', got {m!r}")
    return MAPPINGS[m]


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def version() -> int:
    return load().gocp_version()


def phase_trace(ctx: "Context", n_rows: int) -> np.ndarray:
    """The energy+screen launch's phase timestamps (gocp_phase_trace): an
    (n_rows, 6) uint64 array of 100 MHz clock values per workgroup, from the
    measurement build only (GocpError ENOTSUP otherwise)."""
    out = np.zeros((int(n_rows), 6), dtype=np.uint64)
    nph = C.c_int32()
    check(load().gocp_phase_trace(ctx.handle, out.ctypes.data_as(C.POINTER(C.c_uint64)), int(n_rows),
                                  C.byref(nph)))
    return out[:, :nph.value]


class Hamiltonian:
    """Handle of a folded Pauli-sum Hamiltonian (host object, uploaded on use)."""

    def __init__(self, handle):
        self._h = handle
        lib = load()
        self._free = lib.gocp_ham_free      # kept: module globals may be gone at exit
        nq, nt, nc = C.c_int32(), C.c_int64(), C.c_int32()
        check(lib.gocp_ham_info(self._h, C.byref(nq), C.byref(nt), C.byref(nc)))
        self.n_qubits, self.n_terms, self.n_classes = nq.value, nt.value, nc.value

    @property
    def handle(self):
        return self._h

    def terms(self):
        """(x, z, c) arrays sorted by (x, z): folded coefficients."""
        n = self.n_terms
        x = np.zeros(n, dtype=np.uint32)
        z = np.zeros(n, dtype=np.uint32)
        c = np.zeros(n, dtype=np.float64)
        check(load().gocp_ham_terms(self._h, n, _ptr(x, C.c_uint32), _ptr(z, C.c_uint32),
                                    _ptr(c, C.c_double)))
        return x, z, c

    def __del__(self):
        h, self._h = getattr(self, "_h", None), None
        if h:
            self._free(h)


class Pool:
    """Handle of an operator pool with its GOCP partition (host object)."""

    def __init__(self, handle):
        self._h = handle
        lib = load()
        self._free = lib.gocp_pool_free
        nq, m, s = C.c_int32(), C.c_int32(), C.c_int32()
        check(lib.gocp_pool_info(self._h, C.byref(nq), C.byref(m), C.byref(s)))
        self.n_qubits, self.n_ops, self.n_strings = nq.value, m.value, s.value

    @property
    def handle(self):
        return self._h

    def op(self, k: int):
        """(kind, indices, xmask) of operator k; indices padded with -1."""
        kind = C.c_int32()
        idx = (C.c_int32 * 4)()
        xm = C.c_uint32()
        check(load().gocp_pool_op(self._h, k, C.byref(kind), idx, C.byref(xm)))
        return kind.value, tuple(i for i in idx if i >= 0), xm.value

    def strings(self):
        """(offsets[M+1], xmask per op [M], z[S], c[S])."""
        off = np.zeros(self.n_ops + 1, dtype=np.int32)
        z = np.zeros(self.n_strings, dtype=np.uint32)
        c = np.zeros(self.n_strings, dtype=np.float64)
        check(load().gocp_pool_strings(self._h, _ptr(off, C.c_int32), _ptr(z, C.c_uint32),
                                       _ptr(c, C.c_double)))
        xm = np.array([self.op(k)[2] for k in range(self.n_ops)], dtype=np.uint32)
        return off, xm, z, c

    def degrees(self):
        ne = C.c_int64()
        deg = np.zeros(self.n_ops, dtype=np.int32)
        check(load().gocp_conflict_degrees(self._h, C.byref(ne), _ptr(deg, C.c_int32)))
        return ne.value, deg

    def __del__(self):
        h, self._h = getattr(self, "_h", None), None
        if h:
            self._free(h)


def pauli_hamiltonian_load(h1, eri, e_core: float, mapping) -> Hamiltonian:
    h1 = _f64(h1)
    eri = _f64(eri)
    n = h1.shape[0]
    if h1.shape != (n, n) or eri.shape != (n, n, n, n):
        raise ValueError("h1 must be (n, n) and eri (n, n, n, n)")
    out = C.c_void_p()
    check(load().pauli_hamiltonian_load(n, _ptr(h1, C.c_double), _ptr(eri, C.c_double),
                                        float(e_core), _mapping(mapping), C.byref(out)))
    return Hamiltonian(out)


def pauli_hamiltonian_load_terms(n_qubits: int, x, z, c) -> Hamiltonian:
    x = np.ascontiguousarray(x, dtype=np.uint32)
    z = np.ascontiguousarray(z, dtype=np.uint32)
    c = _f64(c)
    out = C.c_void_p()
    check(load().pauli_hamiltonian_load_terms(n_qubits, len(x), _ptr(x, C.c_uint32),
                                              _ptr(z, C.c_uint32), _ptr(c, C.c_double),
                                              C.byref(out)))
    return Hamiltonian(out)


def pool_build(n_qubits: int, n_electrons: int, mapping) -> Pool:
    out = C.c_void_p()
    check(load().pool_build(n_qubits, n_electrons, _mapping(mapping), C.byref(out)))
    return Pool(out)


def pool_build_pauli(n_qubits: int, n_electrons: int, mapping) -> Pool:
    """One operator per string of the pool_build generators, unit coefficients."""
    out = C.c_void_p()
    check(load().pool_build_pauli(n_qubits, n_electrons, _mapping(mapping), C.byref(out)))
    return Pool(out)


def gocp_partition(pool: Pool):
    """(family_of[M], n_families, order[M]) of Algorithm 1."""
    fam = np.zeros(pool.n_ops, dtype=np.int32)
    order = np.zeros(pool.n_ops, dtype=np.int32)
    k = C.c_int32()
    check(load().gocp_partition(pool.handle, _ptr(fam, C.c_int32), C.byref(k),
                                _ptr(order, C.c_int32)))
    return fam, k.value, order


def hf_index(n_qubits: int, n_electrons: int, mapping) -> int:
    out = C.c_uint64()
    check(load().gocp_hf_index(n_qubits, n_electrons, _mapping(mapping), C.byref(out)))
    return out.value


def basis_occupation(n_qubits: int, mapping, index: int) -> int:
    """Spin-orbital occupations (bit j) of a basis index under the encoding."""
    out = C.c_uint64()
    check(load().gocp_basis_occupation(n_qubits, _mapping(mapping), int(index), C.byref(out)))
    return out.value


# ---------------------------------------------------------------- device side

def _state(psi, n_qubits: int):
    """Pointer and dtype code of a state tensor of 2^n_qubits amplitudes.

    The C ABI receives a bare device pointer and cannot see the buffer's
    length, so the length is checked here, before any launch."""
    import torch
    if not isinstance(psi, torch.Tensor) or not psi.is_cuda:
        raise ValueError("state must be a device tensor")
    if not psi.is_contiguous():
        raise ValueError("state must be contiguous")
    if psi.dtype == torch.complex128:
        code = C128
    elif psi.dtype == torch.complex64:
        code = C64
    else:
        raise ValueError("state must be complex128 or complex64")
    if not 1 <= int(n_qubits) <= 30 or psi.numel() != (1 << int(n_qubits)):
        raise ValueError(f"state has {psi.numel()} amplitudes, expected 2^{n_qubits}")
    return C.c_void_p(psi.data_ptr()), code


def _device_f64(out, n_min: int, what: str):
    """Pointer of a contiguous float64 device tensor holding at least n_min values."""
    import torch
    if (not isinstance(out, torch.Tensor) or not out.is_cuda or out.dtype != torch.float64
            or not out.is_contiguous() or out.numel() < n_min):
        raise ValueError(f"{what} must be a contiguous float64 device tensor of >= {n_min} values")
    return C.cast(C.c_void_p(out.data_ptr()), C.POINTER(C.c_double))


class Context:
    """A device context bound to a HIP device and stream (torch's current one by default)."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(device)
        sp = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream or 0)
        self._c = C.c_void_p()
        self._free = load().gocp_ctx_destroy
        check(load().gocp_ctx_create(device, C.c_void_p(sp), C.byref(self._c)))
        self.device = device

    @property
    def handle(self):
        return self._c

    def set_stream(self, stream):
        sp = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream or 0)
        check(load().gocp_ctx_set_stream(self._c, C.c_void_p(sp)))

    def synchronize(self):
        check(load().gocp_ctx_synchronize(self._c))

    def close(self):
        c, self._c = getattr(self, "_c", None), None
        if c:
            self._free(c)

    def __del__(self):
        self.close()


def state_basis(ctx: Context, n_qubits: int, index: int, psi):
    p, dt = _state(psi, n_qubits)
    check(load().gocp_state_basis(ctx.handle, n_qubits, index, p, dt))


def state_hf(ctx: Context, n_qubits: int, n_electrons: int, mapping, psi):
    """The encoded Hartree-Fock reference into psi."""
    p, dt = _state(psi, n_qubits)
    check(load().gocp_state_hf(ctx.handle, n_qubits, n_electrons, _mapping(mapping), p, dt))


def sector_weight(ctx: Context, n_qubits: int, n_electrons: int, mapping, psi) -> float:
    """Weight of psi inside the (n_electrons, S_z = 0) sector, decoded through the encoding."""
    p, dt = _state(psi, n_qubits)
    w = C.c_double()
    check(load().gocp_sector_weight(ctx.handle, n_qubits, n_electrons, _mapping(mapping), p, dt, C.byref(w)))
    return w.value


def energy(ctx: Context, ham: Hamiltonian, psi) -> float:
    p, dt = _state(psi, ham.n_qubits)
    e = C.c_double()
    check(load().energy(ctx.handle, ham.handle, p, dt, C.byref(e)))
    return e.value


def apply_hamiltonian(ctx: Context, ham: Hamiltonian, psi, sigma, want_energy: bool = True):
    import torch
    if (not isinstance(sigma, torch.Tensor) or sigma.dtype != torch.complex128 or not sigma.is_cuda
            or not sigma.is_contiguous() or sigma.numel() != (1 << ham.n_qubits)):
        raise ValueError(f"sigma must be a contiguous complex128 device tensor of 2^{ham.n_qubits} values")
    p, dt = _state(psi, ham.n_qubits)
    e = C.c_double()
    check(load().gocp_apply_hamiltonian(ctx.handle, ham.handle, p, dt, C.c_void_p(sigma.data_ptr()),
                                        C.byref(e) if want_energy else None))
    return e.value if want_energy else None


def pool_gradients(ctx: Context, ham: Hamiltonian, pool: Pool, psi, out=None):
    """Gradients of every pool operator; host numpy array, or into a device tensor `out`."""
    if ham.n_qubits != pool.n_qubits:
        raise ValueError(f"Hamiltonian has {ham.n_qubits} qubits, pool {pool.n_qubits}")
    p, dt = _state(psi, ham.n_qubits)
    if out is None:
        g = np.zeros(pool.n_ops, dtype=np.float64)
        check(load().pool_gradients(ctx.handle, ham.handle, pool.handle, p, dt,
                                    _ptr(g, C.c_double), 0))
        return g
    check(load().pool_gradients(ctx.handle, ham.handle, pool.handle, p, dt,
                                _device_f64(out, pool.n_ops, "out"), 1))
    return out


def pool_gradients_noalloc(ctx: Context, ham: Hamiltonian, pool: Pool, psi, out):
    """pool_gradients into the device tensor `out` without any device
    allocation (fixed library workspace; the tables must already be resident)."""
    if ham.n_qubits != pool.n_qubits:
        raise ValueError(f"Hamiltonian has {ham.n_qubits} qubits, pool {pool.n_qubits}")
    p, dt = _state(psi, ham.n_qubits)
    check(load().pool_gradients_noalloc(ctx.handle, ham.handle, pool.handle, p, dt,
                                        _device_f64(out, pool.n_ops, "out")))
    return out


def taylor5_apply(ctx: Context, pool: Pool, k: int, theta: float, psi) -> int:
    p, dt = _state(psi, pool.n_qubits)
    s = C.c_int32()
    check(load().taylor5_apply(ctx.handle, pool.handle, k, float(theta), p, dt, C.byref(s)))
    return s.value


def taylor5_apply_family(ctx: Context, pool: Pool, ops, thetas, psi):
    """GOCP multi-operator step over 1-4 operators of one family; substeps per operator."""
    o = np.ascontiguousarray(ops, dtype=np.int32)
    th = _f64(thetas)
    if len(o) != len(th):
        raise ValueError("one angle per operator")
    p, dt = _state(psi, pool.n_qubits)
    ns = np.zeros(len(o), dtype=np.int32)
    check(load().taylor5_apply_family(ctx.handle, pool.handle, len(o), _ptr(o, C.c_int32),
                                      _ptr(th, C.c_double), p, dt, _ptr(ns, C.c_int32)))
    return ns


class _Record:
    """Caller-side arrays of one gocp_adapt_result."""

    def __init__(self, max_iter: int):
        n = max_iter
        self.e = np.zeros(n + 1)
        self.ops = np.zeros(max(n, 1), dtype=np.int32)
        self.th = np.zeros(max(n, 1))
        self.gn = np.zeros(n + 1)
        self.gm = np.zeros(n + 1)
        self.ns = np.zeros(max(n, 1), dtype=np.int32)
        self.res = AdaptResult(0, 0, _ptr(self.e, C.c_double), _ptr(self.ops, C.c_int32),
                               _ptr(self.th, C.c_double), _ptr(self.gn, C.c_double),
                               _ptr(self.gm, C.c_double), _ptr(self.ns, C.c_int32))

    def as_dict(self):
        k = self.res.n_iter
        nscr = k + (1 if self.res.converged else 0)
        return dict(n_iter=k, converged=bool(self.res.converged), energies=self.e[:k + 1].copy(),
                    ops=self.ops[:k].tolist(), thetas=self.th[:k].copy(), gnorms=self.gn[:nscr].copy(),
                    gmax=self.gm[:nscr].copy(), substeps=self.ns[:k].tolist())


def adapt_solve(ctx: Context, ham: Hamiltonian, pool: Pool, psi, max_iter: int,
                grad_tol: float = 0.0, use_graph: bool = True, schedule: int = 1):
    """Run ADAPT in place on psi; returns a dict of per-iteration records.

    schedule: amplitudes per lane of the tile kernels (1, 2, 4), plus 256 * 4
    for four workgroups per tile slot in the compacted H v, H w launch
    (complex64 states; 8 otherwise), or 0 to autotune (Batch.schedule reports
    the choice in this encoding).
    """
    if ham.n_qubits != pool.n_qubits:
        raise ValueError(f"Hamiltonian has {ham.n_qubits} qubits, pool {pool.n_qubits}")
    p, dt = _state(psi, ham.n_qubits)
    rec = _Record(max_iter)
    prm = AdaptParams(float(grad_tol), int(max_iter), 1 if use_graph else 0, int(schedule), 0)
    check(load().adapt_solve(ctx.handle, ham.handle, pool.handle, p, dt, C.byref(prm),
                             C.byref(rec.res)))
    return rec.as_dict()


def adapt_reopt_solve(ctx: Context, ham: Hamiltonian, pool: Pool, psi, max_iter: int, grad_tol: float = 0.0,
                      bfgs_gtol: float = 1e-8, bfgs_max_iter: int = 200):
    """ADAPT with every angle re-optimised by BFGS after each appended
    operator; psi (the starting state) receives the final normalised state.
    Returns energies, ops, thetas (final angles), gnorms, BFGS steps and
    evaluations per iteration."""
    if ham.n_qubits != pool.n_qubits:
        raise ValueError(f"Hamiltonian has {ham.n_qubits} qubits, pool {pool.n_qubits}")
    p, dt = _state(psi, ham.n_qubits)
    n = int(max_iter)
    e = np.zeros(n + 1)
    ops = np.zeros(max(n, 1), dtype=np.int32)
    th = np.zeros(max(n, 1))
    gn = np.zeros(n + 1)
    bs = np.zeros(max(n, 1), dtype=np.int32)
    be = np.zeros(max(n, 1), dtype=np.int32)
    res = ReoptResult(0, 0, _ptr(e, C.c_double), _ptr(ops, C.c_int32), _ptr(th, C.c_double),
                      _ptr(gn, C.c_double), _ptr(bs, C.c_int32), _ptr(be, C.c_int32))
    prm = ReoptParams(float(grad_tol), n, int(bfgs_max_iter), float(bfgs_gtol))
    check(load().adapt_reopt_solve(ctx.handle, ham.handle, pool.handle, p, dt, C.byref(prm), C.byref(res)))
    k = res.n_iter
    nscr = k + (1 if res.converged else 0)
    return dict(n_iter=k, converged=bool(res.converged), energies=e[:k + 1].copy(), ops=ops[:k].tolist(),
                thetas=th[:k].copy(), gnorms=gn[:nscr].copy(), bfgs_steps=bs[:k].tolist(),
                bfgs_evals=be[:k].tolist())


class Batch:
    """Lock-step batch of ADAPT instances (gocp_batch_*)."""

    def __init__(self, ctx: Context, hams, pools, psis, max_iter: int, grad_tol: float = 0.0,
                 use_graph: bool = True, schedule: int = 0):
        n = len(psis)
        if not (len(hams) == len(pools) == n) or n == 0:
            raise ValueError("hams, pools and psis must have the same non-zero length")
        dts = set()
        ptrs = []
        for t, h, q in zip(psis, hams, pools):
            if h.n_qubits != q.n_qubits:
                raise ValueError(f"Hamiltonian has {h.n_qubits} qubits, pool {q.n_qubits}")
            p_, dt = _state(t, h.n_qubits)
            ptrs.append(p_.value)
            dts.add(dt)
        if len(dts) != 1:
            raise ValueError("all states of a batch must share one dtype")
        self.dtype = dts.pop()
        self._keep = (list(hams), list(pools), list(psis))
        H = (C.c_void_p * n)(*[h.handle.value for h in hams])
        P = (C.c_void_p * n)(*[q.handle.value for q in pools])
        S = (C.c_void_p * n)(*ptrs)
        self.max_iter = max_iter
        self.n = n
        prm = AdaptParams(float(grad_tol), int(max_iter), 1 if use_graph else 0, int(schedule), 0)
        self._b = C.c_void_p()
        self._ctx = ctx                     # the context outlives the batch
        self._free = load().gocp_batch_destroy
        check(load().gocp_batch_create(ctx.handle, n, H, P, S, self.dtype, C.byref(prm),
                                       C.byref(self._b)))

    def step(self, n_iter: int):
        check(load().gocp_batch_step(self._b, int(n_iter)))

    STEP_KERNELS = ("k_line_vw", "k_line_hvw", "k_taylor5", "k_energy_screen", "k_screen_sum1")

    def step_timed(self, n_iter: int, kernel: int, every: int = 1):
        """n_iter iterations with HIP events around the launch of one of
        STEP_KERNELS in every `every`-th iteration; returns (total ms, mean ms
        of the sampled launches)."""
        tot, k = C.c_double(), C.c_double()
        check(load().gocp_batch_step_timed(self._b, int(n_iter), int(kernel), int(every), C.byref(tot),
                                           C.byref(k)))
        return tot.value, k.value

    def run(self):
        check(load().gocp_batch_run(self._b))

    def poll(self) -> int:
        a = C.c_int32()
        check(load().gocp_batch_poll(self._b, C.byref(a)))
        return a.value

    def result(self, i: int):
        rec = _Record(self.max_iter)
        check(load().gocp_batch_result(self._b, int(i), C.byref(rec.res)))
        return rec.as_dict()

    @property
    def schedule(self) -> int:
        r = C.c_int32()
        check(load().gocp_batch_schedule(self._b, C.byref(r)))
        return r.value

    def time_kernel(self, which: int, n_launch: int) -> float:
        """Mean duration in ms of launch `which` (gocp_batch_time_kernel: 0 energy and screen partials
        with a fresh H psi, 1 H v / H w of the line search, 2 the partials with sigma carried, 3 the
        reduction of the partials)."""
        ms = C.c_double()
        check(load().gocp_batch_time_kernel(self._b, int(which), int(n_launch), C.byref(ms)))
        return ms.value

    def close(self):
        b, self._b = getattr(self, "_b", None), None
        if b:
            self._free(b)

    def __del__(self):
        self.close()


def request_footprint(ham: Hamiltonian, pool: Pool, max_iter: int, dtype: int = C64) -> int:
    """Device bytes one serving request occupies while admitted (its arena block)."""
    out = C.c_int64()
    check(load().gocp_request_bytes(ham.handle, pool.handle, int(max_iter), int(dtype), C.byref(out)))
    return out.value


class Server:
    """Continuous-batching ADAPT server (gocp_server_*): submit, then poll."""

    def __init__(self, ctx: Context, hbm_budget_bytes: int, max_slots: int, dtype: int = C64,
                 iters_per_step: int = 4, amps_per_lane: int = 1):
        self._s = C.c_void_p()
        self._ctx = ctx
        self._free = load().gocp_server_destroy
        check(load().gocp_server_create(ctx.handle, int(hbm_budget_bytes), int(max_slots), int(dtype),
                                        int(iters_per_step), int(amps_per_lane), C.byref(self._s)))
        self._keep = {}        # ticket -> (ham, pool, max_iter): alive until polled

    def submit(self, ham: Hamiltonian, pool: Pool, max_iter: int, grad_tol: float) -> int:
        t = C.c_uint64()
        check(load().gocp_server_submit(self._s, ham.handle, pool.handle, int(max_iter),
                                        float(grad_tol), C.byref(t)))
        self._keep[t.value] = (ham, pool, int(max_iter))
        return t.value

    def poll(self, ticket: int):
        """None while pending; else (status, record dict or None, info dict)."""
        ham, pool, max_iter = self._keep[ticket]
        rec = _Record(max_iter)
        info = RequestInfo()
        st = load().gocp_server_poll(self._s, ticket, C.byref(rec.res), C.byref(info))
        if st == GOCP_EBUSY:
            return None
        del self._keep[ticket]
        inf = dict(status=info.status, n_qubits=info.n_qubits, t_submit_ns=info.t_submit_ns,
                   t_admit_ns=info.t_admit_ns, t_done_ns=info.t_done_ns)
        return st, (rec.as_dict() if st == 0 else None), inf

    def stats(self):
        a, q = C.c_int32(), C.c_int32()
        c, b, n = C.c_int64(), C.c_int64(), C.c_int64()
        check(load().gocp_server_stats(self._s, C.byref(a), C.byref(q), C.byref(c), C.byref(b),
                                       C.byref(n)))
        return dict(active=a.value, queued=q.value, completed=c.value, bytes_in_use=b.value,
                    steps=n.value)

    def close(self):
        s, self._s = getattr(self, "_s", None), None
        if s:
            self._free(s)

    def __del__(self):
        self.close()
