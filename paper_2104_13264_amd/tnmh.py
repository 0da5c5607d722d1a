"""Thin Python binding of libtnmh.so (include/tnmh.h).

Argument marshalling only: every step of the method runs in the HIP kernels
of the library.  Torch provides device memory and the stream; tensors are
passed by data pointer.  The binding refuses to run without the in-tree
shared object (there is no fallback path).
"""
import ctypes
import os

import torch

FP64, FP32, BF16, FP64_MFMA = 0, 1, 2, 3
PREC = {"fp64": FP64, "fp32": FP32, "bf16": BF16, "fp64_mfma": FP64_MFMA}

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtnmh.so")
_lib = None

_STATUS = {0: "TN_OK", -1: "TN_EINVAL", -2: "TN_ENOMEM", -3: "TN_EHIP",
           -4: "TN_ENONPOS", -5: "TN_ENOCONV", -6: "TN_ESTATE"}


class _Instance(ctypes.Structure):
    _fields_ = [("Lx", ctypes.c_int), ("Ly", ctypes.c_int), ("D", ctypes.c_int),
                ("beta", ctypes.c_double), ("Jh", ctypes.c_void_p), ("Jv", ctypes.c_void_p),
                ("h", ctypes.c_void_p), ("chains", ctypes.c_int)]


class _PeriodicInstance(ctypes.Structure):
    _fields_ = [("Jh", ctypes.c_void_p), ("Jv", ctypes.c_void_p), ("h", ctypes.c_void_p),
                ("beta", ctypes.c_double), ("chains", ctypes.c_int)]


class TNError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


class _Stats(ctypes.Structure):
    _fields_ = [("clamps", ctypes.c_uint64), ("both_nonpos", ctypes.c_uint64),
                ("near_threshold", ctypes.c_uint64), ("accepted", ctypes.c_uint64),
                ("proposed", ctypes.c_uint64), ("degenerate_cuts", ctypes.c_uint64),
                ("logZ", ctypes.c_double), ("env_build_ms", ctypes.c_double),
                ("metropolis_flips", ctypes.c_uint64)]


def lib():
    """Load libtnmh.so once; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2104_13264_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i, d, u64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_uint64
    sig = {
        "tn_create": (i, [ctypes.POINTER(vp), vp]),
        "tn_destroy": (i, [vp]),
        "tn_last_error": (ctypes.c_char_p, [vp]),
        "tn_build_env": (i, [vp, i, i, vp, vp, vp, d, i, i, ctypes.POINTER(d)]),
        "tn_set_env": (i, [vp, i, i, vp, vp, vp, d, i, i, vp, vp, vp, d]),
        "tn_get_env": (i, [vp, vp, vp, vp, ctypes.POINTER(d)]),
        "tn_set_precision": (i, [vp, i]),
        "tn_set_instance": (i, [vp, i]),
        "tn_set_compression": (i, [vp, i]),
        "tn_sample": (i, [vp, i, u64, u64, u64, vp, vp, vp]),
        "tn_sample_noalloc": (i, [vp, i, u64, u64, u64, vp, vp, vp]),
        "tn_eval_logq": (i, [vp, i, vp, vp, vp]),
        "tn_mh_step": (i, [vp, i, u64, u64, vp, vp, vp, vp]),
        "tn_sample_steps": (i, [vp, i, i, u64, u64, u64, vp, vp, vp]),
        "tn_build_env_begin": (i, [vp, i, i, vp, vp, vp, d, i, i]),
        "tn_build_env_rows": (i, [vp, i, ctypes.POINTER(i)]),
        "tn_build_env_end": (i, [vp, ctypes.POINTER(d)]),
        "tn_build_env_multi": (i, [vp, i, vp, i, vp]),
        "tn_mh_step_multi": (i, [vp, u64, u64, vp, vp, vp, vp]),
        "tn_multi_instance": (vp, [vp, i]),
        "tn_graph_begin": (i, [vp]),
        "tn_graph_end_and_replay": (i, [vp, i]),
        "tn_mh_run": (i, [vp, i, i, u64, u64, vp, vp, vp, vp, vp]),
        "tn_mh_accept": (i, [vp, i, u64, u64, vp, vp, vp, vp, vp, vp, vp]),
        "tn_grad": (i, [vp, vp, vp, ctypes.POINTER(d)]),
        "tn_grad_two_sided": (i, [vp, vp, vp, ctypes.POINTER(d)]),
        "tn_logz_frozen": (i, [vp, i, vp, vp, vp, vp, vp]),
        "tn_potts_build_env": (i, [vp, i, i, i, vp, vp, vp, d, i, ctypes.POINTER(d)]),
        "tn_stats": (i, [vp, ctypes.POINTER(_Stats), i]),
        "tn_autotune": (i, [vp, i, i, ctypes.c_char_p, ctypes.POINTER(i), ctypes.POINTER(i)]),
        "tn_autotune_multi": (i, [vp, ctypes.c_char_p, ctypes.POINTER(i)]),
        "tn_metropolis_sweeps": (i, [vp, i, i, u64, u64, vp, vp, vp]),
        "tn_link_overlap": (i, [vp, i, vp, vp, vp]),
        "tn_periodic_setup": (i, [vp, i, i, i, i, i, i, i, vp]),
        "tn_periodic_step": (i, [vp, u64, u64, i, i, vp, vp, vp]),
        "tn_periodic_energy": (i, [vp, vp, vp]),
        "tn_periodic_sweeps": (i, [vp, i, u64, u64, vp, vp]),
        "tn_periodic_link_overlap": (i, [vp, i, vp, vp, vp]),
        "tn_peak_probe": (i, [i, ctypes.c_longlong, ctypes.POINTER(d), ctypes.POINTER(d)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def exported_symbols():
    return ["tn_create", "tn_destroy", "tn_last_error", "tn_build_env", "tn_set_env",
            "tn_get_env", "tn_set_precision", "tn_set_instance", "tn_build_env_begin",
            "tn_build_env_rows", "tn_build_env_end", "tn_sample",
            "tn_eval_logq", "tn_mh_step", "tn_mh_accept", "tn_sample_steps", "tn_mh_run",
            "tn_build_env_multi", "tn_mh_step_multi", "tn_multi_instance", "tn_graph_begin",
            "tn_graph_end_and_replay", "tn_grad", "tn_grad_two_sided", "tn_stats",
            "tn_autotune", "tn_autotune_multi", "tn_metropolis_sweeps", "tn_link_overlap",
            "tn_periodic_setup", "tn_periodic_step", "tn_periodic_energy", "tn_periodic_link_overlap",
            "tn_set_compression", "tn_periodic_sweeps", "tn_sample_noalloc", "tn_logz_frozen",
            "tn_potts_build_env", "tn_peak_probe"]


PEAK_KINDS = {"mfma_f32": 0, "mfma_bf16": 1, "mfma_f64": 2, "fma_f64": 3, "hbm_read": 4, "hbm_copy": 5}


def peak_probe(kind, amount):
    """tn_peak_probe on the current device: (seconds, work) of one timed
    launch of the probe `kind` (a key of PEAK_KINDS); amount is iterations
    for the compute probes, buffer bytes for the memory ones."""
    if not torch.cuda.is_available():
        raise TNError("no GPU: the probes run HIP kernels")
    sec, work = ctypes.c_double(), ctypes.c_double()
    rc = lib().tn_peak_probe(PEAK_KINDS[kind], int(amount), ctypes.byref(sec), ctypes.byref(work))
    if rc != 0:
        raise TNError(f"tn_peak_probe({kind}, {amount}) failed with code {rc}")
    return sec.value, work.value


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _dev64(x, device):
    if x is None:
        return None
    t = torch.as_tensor(x, dtype=torch.float64, device=device)
    return t.contiguous()


class Sampler:
    """One library context: an environment stack and its samplers."""

    def __init__(self, device=None, stream=None):
        if not torch.cuda.is_available():
            raise RuntimeError("the TNMH library needs a HIP device")
        self.device = torch.device(device or f"cuda:{torch.cuda.current_device()}")
        self.stream = stream or torch.cuda.current_stream(self.device)
        self._ctx = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            self._check(lib().tn_create(ctypes.byref(self._ctx),
                                        ctypes.c_void_p(self.stream.cuda_stream)))
        self.Lx = self.Ly = self.D = None
        self.beta = None
        self.d = None   # number of values of a Potts context

    # -- plumbing -----------------------------------------------------------
    def _check(self, rc):
        if rc != 0:
            msg = lib().tn_last_error(self._ctx).decode() if self._ctx else ""
            raise TNError(rc, msg)

    def close(self):
        if self._ctx:
            lib().tn_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- environments -------------------------------------------------------
    def build_env(self, Jh, Jv, h, beta, D, prec=FP64, progress=None, rows_per_call=16):
        """Build the boundary-MPS environments; returns ln Z~.  With
        progress(rows_done, rows_total), the rows are built in chunks of
        rows_per_call and progress is called after each chunk."""
        Jh, Jv, h = (_dev64(x, self.device) for x in (Jh, Jv, h))
        Ly, Lx = Jv.shape[0] + 1, Jh.shape[1] + 1
        self._keep = (Jh, Jv, h)
        logZ = ctypes.c_double()
        if progress is None:
            self._check(lib().tn_build_env(self._ctx, Lx, Ly, _ptr(Jh), _ptr(Jv), _ptr(h),
                                           float(beta), int(D), int(prec), ctypes.byref(logZ)))
        else:
            self._check(lib().tn_build_env_begin(self._ctx, Lx, Ly, _ptr(Jh), _ptr(Jv), _ptr(h),
                                                 float(beta), int(D), int(prec)))
            left = ctypes.c_int(Ly - 1)
            while left.value > 0:
                self._check(lib().tn_build_env_rows(self._ctx, int(rows_per_call),
                                                    ctypes.byref(left)))
                progress(Ly - 1 - left.value, Ly - 1)
            self._check(lib().tn_build_env_end(self._ctx, ctypes.byref(logZ)))
        self.Lx, self.Ly, self.D, self.beta = Lx, Ly, int(D), float(beta)
        self.d = None
        return logZ.value

    def potts_build_env(self, Jh, Jv, h, beta, D, d):
        """Environments of a q-state Potts model with d values
        (tn_potts_build_env; h: [Ly][Lx][d] or None); returns ln Z~.  The
        sampling calls then draw value configurations 0..d-1."""
        Jh, Jv, h = (_dev64(x, self.device) for x in (Jh, Jv, h))
        Ly, Lx = Jv.shape[0] + 1, Jh.shape[1] + 1
        self._keep = (Jh, Jv, h)
        logZ = ctypes.c_double()
        self._check(lib().tn_potts_build_env(self._ctx, Lx, Ly, int(d), _ptr(Jh), _ptr(Jv), _ptr(h),
                                             float(beta), int(D), ctypes.byref(logZ)))
        self.Lx, self.Ly, self.D, self.beta, self.d = Lx, Ly, int(D), float(beta), int(d)
        return logZ.value

    def set_env(self, Jh, Jv, h, beta, D, env, dims, ell, logZ, prec=FP64):
        """Install environments given as host arrays (layout of tn_set_env)."""
        import numpy as np
        Jh, Jv, h = (_dev64(x, self.device) for x in (Jh, Jv, h))
        Ly, Lx = Jv.shape[0] + 1, Jh.shape[1] + 1
        env = np.ascontiguousarray(env, dtype=np.float64)
        dims = np.ascontiguousarray(dims, dtype=np.int32)
        ell = np.ascontiguousarray(ell, dtype=np.float64)
        self._check(lib().tn_set_env(self._ctx, Lx, Ly, _ptr(Jh), _ptr(Jv), _ptr(h),
                                     float(beta), int(D), int(prec),
                                     env.ctypes.data_as(ctypes.c_void_p),
                                     dims.ctypes.data_as(ctypes.c_void_p),
                                     ell.ctypes.data_as(ctypes.c_void_p), float(logZ)))
        self.Lx, self.Ly, self.D, self.beta = Lx, Ly, int(D), float(beta)
        self.d = None

    def get_env(self):
        """Return (env [(Ly-1)][Lx][D][2][D], dims [(Ly-1)][Lx+1], ell, logZ)."""
        import numpy as np
        Lx, Ly, D = self.Lx, self.Ly, self.D
        env = np.zeros((max(Ly - 1, 0), Lx, D, 2, D))
        dims = np.zeros((max(Ly - 1, 0), Lx + 1), dtype=np.int32)
        ell = np.zeros(max(Ly - 1, 0))
        lz = ctypes.c_double()
        self._check(lib().tn_get_env(self._ctx, env.ctypes.data_as(ctypes.c_void_p),
                                     dims.ctypes.data_as(ctypes.c_void_p),
                                     ell.ctypes.data_as(ctypes.c_void_p), ctypes.byref(lz)))
        return env, dims, ell, lz.value

    def set_precision(self, prec):
        self._check(lib().tn_set_precision(self._ctx, int(prec)))

    def set_instance(self, inst):
        self._check(lib().tn_set_instance(self._ctx, int(inst)))

    def set_compression(self, fit_sweeps):
        """0: successive SVD; n > 0: successive SVD then n two-site variational
        sweeps, for the builds that follow (tn_set_compression)."""
        self._check(lib().tn_set_compression(self._ctx, int(fit_sweeps)))

    # -- sampling -----------------------------------------------------------
    def empty_batch(self, batch):
        return (torch.empty((batch, self.Ly, self.Lx), dtype=torch.int8, device=self.device),
                torch.empty(batch, dtype=torch.float64, device=self.device),
                torch.empty(batch, dtype=torch.float64, device=self.device))

    def sample(self, batch, seed, step=0, first_id=0, out=None):
        s, lq, E = out if out is not None else self.empty_batch(batch)
        self._check(lib().tn_sample(self._ctx, int(batch), int(seed), int(step), int(first_id),
                                    _ptr(s), _ptr(lq), _ptr(E)))
        return s, lq, E

    def sample_noalloc(self, batch, seed, step=0, first_id=0, out=None):
        """sample() through tn_sample_noalloc: the library allocates nothing
        (the caller passes the output buffers in `out`)."""
        s, lq, E = out if out is not None else self.empty_batch(batch)
        self._check(lib().tn_sample_noalloc(self._ctx, int(batch), int(seed), int(step), int(first_id),
                                            _ptr(s), _ptr(lq), _ptr(E)))
        return s, lq, E

    def sample_steps(self, chains, nsteps, seed, step0=0, first_id=0, out=None):
        """Proposals of nsteps MH steps at once: tensors [nsteps][chains]..."""
        if out is None:
            out = (torch.empty((nsteps, chains, self.Ly, self.Lx), dtype=torch.int8,
                               device=self.device),
                   torch.empty((nsteps, chains), dtype=torch.float64, device=self.device),
                   torch.empty((nsteps, chains), dtype=torch.float64, device=self.device))
        s, lq, E = out
        self._check(lib().tn_sample_steps(self._ctx, int(chains), int(nsteps), int(seed),
                                          int(step0), int(first_id), _ptr(s), _ptr(lq), _ptr(E)))
        return s, lq, E

    def eval_logq(self, spins):
        spins = torch.as_tensor(spins, dtype=torch.int8, device=self.device).contiguous()
        B = spins.shape[0]
        lq = torch.empty(B, dtype=torch.float64, device=self.device)
        E = torch.empty(B, dtype=torch.float64, device=self.device)
        self._check(lib().tn_eval_logq(self._ctx, B, _ptr(spins), _ptr(lq), _ptr(E)))
        return lq, E

    def init_state(self, chains, spins=None):
        """Chains in the given configurations, by default all up (Ising) or
        all value 0 (Potts), with ln q and H from tn_eval_logq."""
        if spins is None:
            fill = torch.zeros if self.d else torch.ones
            spins = fill((chains, self.Ly, self.Lx), dtype=torch.int8, device=self.device)
        spins = torch.as_tensor(spins, dtype=torch.int8, device=self.device).contiguous().clone()
        lq, E = self.eval_logq(spins)
        acc = torch.zeros(spins.shape[0], dtype=torch.uint8, device=self.device)
        return dict(spins=spins, logq=lq, energy=E, accepted=acc)

    def mh_step(self, state, seed, step):
        C = state["spins"].shape[0]
        self._check(lib().tn_mh_step(self._ctx, C, int(seed), int(step), _ptr(state["spins"]),
                                     _ptr(state["logq"]), _ptr(state["energy"]),
                                     _ptr(state["accepted"])))
        return state["accepted"]

    # -- batched uneven instances -----------------------------------------
    def build_env_multi(self, instances, prec=FP32):
        """instances: sequence of dicts with Jh, Jv, h (or None), beta, D, chains.
        Returns ln Z~ per instance; self.instance(i) gives instance i."""
        n = len(instances)
        arr = (_Instance * n)()
        keep = []
        for k, it in enumerate(instances):
            Jh, Jv, h = (_dev64(it.get(x), self.device) for x in ("Jh", "Jv", "h"))
            keep.append((Jh, Jv, h))
            Ly, Lx = Jv.shape[0] + 1, Jh.shape[1] + 1
            arr[k] = _Instance(Lx, Ly, int(it["D"]), float(it["beta"]),
                               Jh.data_ptr() if Jh.numel() else None,
                               Jv.data_ptr() if Jv.numel() else None,
                               h.data_ptr() if h is not None else None, int(it["chains"]))
        self._keep_multi = keep
        lz = (ctypes.c_double * n)()
        self._check(lib().tn_build_env_multi(self._ctx, n, arr, int(prec), lz))
        self._multi = [(arr[k].Lx, arr[k].Ly, arr[k].D, arr[k].beta) for k in range(n)]
        return list(lz)

    def instance(self, i):
        """Instance i of the batched context (a borrowed Sampler)."""
        p = lib().tn_multi_instance(self._ctx, int(i))
        if not p:
            raise TNError(-1, f"no instance {i}")
        Lx, Ly, D, beta = self._multi[i]
        return _BorrowedSampler(self, p, Lx, Ly, D, beta)

    def mh_step_multi(self, states, seed, step):
        n = len(states)
        P = ctypes.c_void_p * n
        sp = P(*[s["spins"].data_ptr() for s in states])
        lq = P(*[s["logq"].data_ptr() for s in states])
        en = P(*[s["energy"].data_ptr() for s in states])
        ac = P(*[s["accepted"].data_ptr() for s in states])
        self._check(lib().tn_mh_step_multi(self._ctx, int(seed), int(step), sp, lq, en, ac))

    def graph_begin(self):
        self._check(lib().tn_graph_begin(self._ctx))

    def graph_end_and_replay(self, n_replays):
        self._check(lib().tn_graph_end_and_replay(self._ctx, int(n_replays)))

    def mh_run(self, state, seed, step0, nsteps, energy_series=True):
        """nsteps MH steps; returns (accepted [nsteps][chains], energies or None)."""
        C = state["spins"].shape[0]
        acc = torch.empty((nsteps, C), dtype=torch.uint8, device=self.device)
        es = (torch.empty((nsteps, C), dtype=torch.float64, device=self.device)
              if energy_series else None)
        self._check(lib().tn_mh_run(self._ctx, C, int(nsteps), int(seed), int(step0),
                                    _ptr(state["spins"]), _ptr(state["logq"]),
                                    _ptr(state["energy"]), _ptr(acc),
                                    _ptr(es) if es is not None else None))
        return acc, es

    def metropolis_sweeps(self, state, nsweeps, seed, step):
        """nsweeps single-spin-flip Metropolis sweeps of every chain in place
        (tn_metropolis_sweeps); ln q and the energy are re-evaluated."""
        C = state["spins"].shape[0]
        self._check(lib().tn_metropolis_sweeps(self._ctx, C, int(nsweeps), int(seed), int(step),
                                               _ptr(state["spins"]), _ptr(state["logq"]),
                                               _ptr(state["energy"])))
        return state

    def link_overlap(self, a, b):
        """sum over the bonds of a_i a_j b_i b_j per configuration pair
        (tn_link_overlap); a, b: int8 [n][Ly][Lx] on the device."""
        a = torch.as_tensor(a, dtype=torch.int8, device=self.device).contiguous()
        b = torch.as_tensor(b, dtype=torch.int8, device=self.device).contiguous()
        q = torch.empty(a.shape[0], dtype=torch.int32, device=self.device)
        self._check(lib().tn_link_overlap(self._ctx, a.shape[0], _ptr(a), _ptr(b), _ptr(q)))
        return q

    # -- periodic boundaries by frozen lines ------------------------------
    def periodic_setup(self, instances, Lx, Ly, wrap_x, wrap_y, D, prec=FP32):
        """instances: dicts with Jh, Jv, h (or None), beta, chains; couplings
        in the periodic layout of tn_periodic_setup."""
        n = len(instances)
        arr = (_PeriodicInstance * n)()
        keep = []
        for k, it in enumerate(instances):
            Jh, Jv, h = (_dev64(it.get(x), self.device) for x in ("Jh", "Jv", "h"))
            keep.append((Jh, Jv, h))
            arr[k] = _PeriodicInstance(Jh.data_ptr() if Jh.numel() else None,
                                       Jv.data_ptr() if Jv.numel() else None,
                                       h.data_ptr() if h is not None else None,
                                       float(it["beta"]), int(it["chains"]))
        self._check(lib().tn_periodic_setup(self._ctx, int(Lx), int(Ly), int(bool(wrap_x)),
                                            int(bool(wrap_y)), int(D), int(prec), n, arr))
        self._periodic = (int(Lx), int(Ly), sum(int(it["chains"]) for it in instances))
        return self

    def periodic_step(self, spins, seed, step, cut_row, cut_col, energy=None, accepted=None):
        """One TNMH step of every chain with the given cut; spins (int8
        [chains][Ly][Lx] on the device) are updated in place.  Returns the
        periodic energies and the accept flags."""
        if spins.dtype != torch.int8 or not spins.is_contiguous() or spins.device != self.device:
            raise ValueError("spins must be a contiguous int8 tensor on the context's device")
        T = spins.shape[0]
        if energy is None:
            energy = torch.empty(T, dtype=torch.float64, device=self.device)
        if accepted is None:
            accepted = torch.empty(T, dtype=torch.uint8, device=self.device)
        self._check(lib().tn_periodic_step(self._ctx, int(seed), int(step), int(cut_row), int(cut_col),
                                           _ptr(spins), _ptr(energy), _ptr(accepted)))
        return energy, accepted

    def periodic_sweeps(self, spins, nsweeps, seed, step):
        """nsweeps Metropolis sweeps of every chain on the periodic lattice,
        in place (tn_periodic_sweeps); returns the periodic energies."""
        if spins.dtype != torch.int8 or not spins.is_contiguous() or spins.device != self.device:
            raise ValueError("spins must be a contiguous int8 tensor on the context's device")
        E = torch.empty(spins.shape[0], dtype=torch.float64, device=self.device)
        self._check(lib().tn_periodic_sweeps(self._ctx, int(nsweeps), int(seed), int(step), _ptr(spins), _ptr(E)))
        return E

    def periodic_energy(self, spins):
        spins = torch.as_tensor(spins, dtype=torch.int8, device=self.device).contiguous()
        E = torch.empty(spins.shape[0], dtype=torch.float64, device=self.device)
        self._check(lib().tn_periodic_energy(self._ctx, _ptr(spins), _ptr(E)))
        return E

    def periodic_link_overlap(self, a, b):
        a = torch.as_tensor(a, dtype=torch.int8, device=self.device).contiguous()
        b = torch.as_tensor(b, dtype=torch.int8, device=self.device).contiguous()
        q = torch.empty(a.shape[0], dtype=torch.int32, device=self.device)
        self._check(lib().tn_periodic_link_overlap(self._ctx, a.shape[0], _ptr(a), _ptr(b), _ptr(q)))
        return q

    def mh_accept(self, proposal, state, seed, step):
        """Acceptance half of an MH step for proposals drawn with sample()."""
        sp, lq, E = proposal
        C = state["spins"].shape[0]
        self._check(lib().tn_mh_accept(self._ctx, C, int(seed), int(step), _ptr(sp), _ptr(lq),
                                       _ptr(E), _ptr(state["spins"]), _ptr(state["logq"]),
                                       _ptr(state["energy"]), _ptr(state["accepted"])))
        return state["accepted"]

    def grad(self, two_sided=False):
        """(dJh, dJv, dbeta): the frozen-truncation derivative of ln Z~
        (tn_grad), or with two_sided=True the two-sided estimate of the
        derivative of ln Z (tn_grad_two_sided)."""
        dJh = torch.zeros((self.Ly, self.Lx - 1), dtype=torch.float64, device=self.device)
        dJv = torch.zeros((self.Ly - 1, self.Lx), dtype=torch.float64, device=self.device)
        db = ctypes.c_double()
        fn = lib().tn_grad_two_sided if two_sided else lib().tn_grad
        self._check(fn(self._ctx, _ptr(dJh), _ptr(dJv), ctypes.byref(db)))
        return dJh, dJv, db.value

    def logz_frozen(self, sets):
        """ln Z~_frozen (tn_logz_frozen) for every (Jh, Jv, h, beta) in `sets`
        with the projectors of the current build.  Returns a list of floats."""
        n = len(sets)
        keep = []
        pj = (ctypes.c_void_p * n)()
        pv = (ctypes.c_void_p * n)()
        ph = (ctypes.c_void_p * n)()
        b = (ctypes.c_double * n)()
        for k, (Jh, Jv, h, beta) in enumerate(sets):
            tJh, tJv = _dev64(Jh, self.device), _dev64(Jv, self.device)
            th = None if h is None else _dev64(h, self.device)
            keep += [tJh, tJv, th]
            pj[k], pv[k] = tJh.data_ptr(), tJv.data_ptr()
            ph[k] = None if th is None else th.data_ptr()
            b[k] = float(beta)
        out = (ctypes.c_double * n)()
        self._check(lib().tn_logz_frozen(self._ctx, n, pj, pv, ph, b, out))
        return list(out)

    def autotune(self, chains, max_steps=16, cache=None):
        """Pick the batched sampler's launch variant and the MH steps per
        sampler launch of mh_run by timing them (tn_autotune).  cache: path of
        the JSON file of earlier choices, or None.  Returns (variant, steps)."""
        v, m = ctypes.c_int(), ctypes.c_int()
        self._check(lib().tn_autotune(self._ctx, int(chains), int(max_steps),
                                      os.fsencode(cache) if cache else None,
                                      ctypes.byref(v), ctypes.byref(m)))
        return v.value, m.value

    def autotune_multi(self, cache=None):
        """Pick the launch variant of every sampler group of mh_step_multi by
        timing (tn_autotune_multi).  Returns {(bf16, NT): variant}."""
        out = (ctypes.c_int * 8)()
        self._check(lib().tn_autotune_multi(self._ctx, os.fsencode(cache) if cache else None, out))
        return {(k // 4 == 1, k % 4 + 1): out[k] for k in range(8) if out[k] >= 0}

    def stats(self, reset=False):
        st = _Stats()
        self._check(lib().tn_stats(self._ctx, ctypes.byref(st), 1 if reset else 0))
        return {name: getattr(st, name) for name, _ in _Stats._fields_}


class _BorrowedSampler(Sampler):
    """One instance of a batched context: every single-instance method, on a
    context the batched one owns (close() does not destroy it)."""

    def __init__(self, parent, ptr, Lx, Ly, D, beta):
        self.device = parent.device
        self.stream = parent.stream
        self._ctx = ctypes.c_void_p(ptr)
        self._parent = parent
        self.Lx, self.Ly, self.D, self.beta = Lx, Ly, D, beta
        self.d = None

    def close(self):
        self._ctx = ctypes.c_void_p()


class LogZ(torch.autograd.Function):
    """ln Z~ of the boundary-MPS contraction as a differentiable function of
    the couplings and beta.  The forward builds the environments (tn_build_env,
    fp64).  The backward is one of two derivatives (argument `estimator`):

    "frozen" (default): tn_grad, the adjoint of the contraction with the
        truncation isometries frozen.  It is the exact derivative of the
        frozen contraction, which equals ln Z~ at the build point, and of
        ln Z when nothing was truncated.  With truncation it can be far from
        beta times the bond correlations and minus the energy: on the 128 x 128
        fully frustrated lattice at beta = 1, D = 32, a bulk bond gets 0.897
        where the chain and central differences of the rebuilt ln Z~ give
        0.462, and d/d beta gets 23882 against -<E> = 15070.
    "two_sided": tn_grad_two_sided, every row contracted exactly between the
        top-down and the bottom-up boundaries; on that lattice it agrees with
        the chain (0.462 and 15070.4) and with central differences of the
        rebuilt ln Z~.  It is not the derivative of the frozen contraction.
    """

    @staticmethod
    def forward(ctx, Jh, Jv, beta, D, h=None, estimator="frozen"):
        if estimator not in ("frozen", "two_sided"):
            raise ValueError("estimator must be 'frozen' or 'two_sided'")
        s = Sampler(device=Jh.device)
        b = float(beta.item() if torch.is_tensor(beta) else beta)
        lz = s.build_env(Jh.detach(), Jv.detach(), None if h is None else h.detach(), b, int(D),
                         FP64)
        ctx.sampler = s
        ctx.two_sided = estimator == "two_sided"
        return torch.tensor(lz, dtype=torch.float64, device=Jh.device)

    @staticmethod
    def backward(ctx, g):
        s = ctx.sampler
        dJh, dJv, db = s.grad(two_sided=ctx.two_sided)
        s.close()
        ctx.sampler = None
        g = g.to(torch.float64)
        return g * dJh, g * dJv, g * torch.tensor(db, dtype=torch.float64, device=dJh.device), None, None, None


def log_z(Jh, Jv, beta, D, h=None, estimator="frozen"):
    """Differentiable ln Z~ (see LogZ for the two derivatives `estimator`
    selects); the field h is held fixed."""
    return LogZ.apply(Jh, Jv, beta, D, h, estimator)
