"""ctypes binding of libflb.so (the C ABI in include/flb.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  PyTorch provides device memory and streams.  If the library
has not been built, or no GPU is present, the calls raise; there is no CPU
fallback.
"""

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# FLB_LIB selects another build of the library (the sanitized one, for instance)
LIB_PATH = os.environ.get("FLB_LIB") or os.path.join(HERE, "lib", "libflb.so")

FLB_OK, FLB_EINVAL, FLB_ENOMEM, FLB_EDEVICE, FLB_ESTATE, FLB_ENONFINITE = 0, -1, -2, -3, -4, -5
MODELS = {"D1Q3": 1, "D2Q5": 2, "D3Q7": 3, 1: 1, 2: 2, 3: 3}
NOISE = {"local": 0, "global": 1, "off": 2}
LAWS = {"gauss": 0, "uniform": 1}
KERNELS = {"auto": 0, "plain": 1, "rows": 2, "flat": 3, "resident": 4, "two": 5}
LAYOUTS = {"two": 0, "aa": 1}
SK_SNAPSHOT, SK_SAMPLE, SK_READ, SK_RESET = 0, 1, 2, 3

# exported symbols, in the order include/flb.h declares them
EXPORTS = (
    "flb_version", "flb_last_error", "flb_lattice_constants", "flb_required_bytes",
    "flb_create", "flb_set_populations", "flb_get_populations", "flb_step", "flb_set_check",
    "flb_get_step", "flb_moments", "flb_structure_factor", "flb_set_sampling",
    "flb_set_moment_sampling", "flb_sampled_moments", "flb_set_correlation",
    "flb_correlation", "flb_fourier_amplitudes", "flb_profile", "flb_set_regions", "flb_profile_noalloc",
    "flb_sync",
    "flb_destroy",
    "flb_noise_sample", "flb_gauss_map", "flb_batch_create", "flb_batch_admit", "flb_batch_retire",
    "flb_batch_step", "flb_batch_size", "flb_batch_sync", "flb_batch_destroy",
)


class FlbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"flb error {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [
        ("model", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("n", ctypes.c_int64 * 3), ("theta", ctypes.c_double),
        ("omega", ctypes.c_double * 3), ("seed", ctypes.c_uint64),
        ("noise", ctypes.c_int32), ("noise_law", ctypes.c_int32),
        ("layout", ctypes.c_int32), ("kernel", ctypes.c_int32),
        ("tile_x", ctypes.c_int32), ("tile_rows", ctypes.c_int32),
        ("nt_store", ctypes.c_int32), ("pipeline", ctypes.c_int32),
    ]


class Moments(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_int64), ("nsite", ctypes.c_int64),
        ("mass", ctypes.c_double), ("mass0", ctypes.c_double), ("rho_eq", ctypes.c_double),
        ("sum_f", ctypes.c_double * 7), ("sum_ff", ctypes.c_double * 28),
        ("sum_rho2", ctypes.c_double), ("sum_rho_pos", ctypes.c_double),
        ("n_negative", ctypes.c_int64), ("nonfinite", ctypes.c_int64),
    ]


class BatchOpts(ctypes.Structure):
    _fields_ = [
        ("chunk", ctypes.c_int32), ("use_graph", ctypes.c_int32),
        ("lds_max_bytes", ctypes.c_int32), ("workers", ctypes.c_int32),
        ("item_rows", ctypes.c_int32), ("tiling", ctypes.c_int32),
        ("depth", ctypes.c_int32), ("width", ctypes.c_int32), ("hip_stream", ctypes.c_void_p),
    ]


_lib = None


def load(path=LIB_PATH):
    """Load libflb.so once; raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(
            f"{path} is not built; run `python -m paper_1606_07801_amd.build` first")
    # torch (which allocates the device buffers) ships its own HIP runtime
    # under the same soname as the system one.  Loading torch first makes
    # the library bind to that runtime, so the process holds one HIP runtime;
    # with the system runtime loaded first, device queries in the library
    # can fail while torch still sees the GPU.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    vp, i32, i64, u64, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p
    sig = {
        "flb_version": ([], ctypes.c_int),
        "flb_last_error": ([], ctypes.c_char_p),
        "flb_lattice_constants": ([i32, ctypes.c_double, dp, dp], ctypes.c_int),
        "flb_required_bytes": ([ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_size_t),
                                ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "flb_create": ([ctypes.POINTER(Params), vp, ctypes.c_size_t, vp, ctypes.c_size_t, vp,
                        ctypes.POINTER(vp)], ctypes.c_int),
        "flb_set_populations": ([vp, vp, ctypes.c_int, i64], ctypes.c_int),
        "flb_get_populations": ([vp, vp, ctypes.c_int], ctypes.c_int),
        "flb_step": ([vp, i64], ctypes.c_int),
        "flb_set_check": ([vp, i64], ctypes.c_int),
        "flb_get_step": ([vp, ctypes.POINTER(i64)], ctypes.c_int),
        "flb_moments": ([vp, ctypes.POINTER(Moments)], ctypes.c_int),
        "flb_structure_factor": ([vp, vp, i32, i32, dp], ctypes.c_int),
        "flb_set_sampling": ([vp, i64, vp, i32], ctypes.c_int),
        "flb_set_moment_sampling": ([vp, i64], ctypes.c_int),
        "flb_sampled_moments": ([vp, ctypes.POINTER(Moments), ctypes.POINTER(i64)], ctypes.c_int),
        "flb_set_correlation": ([vp, i64, vp, i32, i32], ctypes.c_int),
        "flb_correlation": ([vp, dp, dp, ctypes.POINTER(i64)], ctypes.c_int),
        "flb_fourier_amplitudes": ([vp, dp], ctypes.c_int),
        "flb_profile": ([vp, i32, dp, dp], ctypes.c_int),
        "flb_set_regions": ([vp, vp, i32, dp, dp], ctypes.c_int),
        "flb_profile_noalloc": ([vp, i32, vp, vp], ctypes.c_int),
        "flb_sync": ([vp], ctypes.c_int),
        "flb_destroy": ([vp], ctypes.c_int),
        "flb_noise_sample": ([i32, i32, i32, u64, i64, i64, i64, vp, vp, vp], ctypes.c_int),
        "flb_gauss_map": ([i32, vp, i64, vp, vp], ctypes.c_int),
        "flb_batch_create": ([ctypes.POINTER(BatchOpts), ctypes.POINTER(vp)], ctypes.c_int),
        "flb_batch_admit": ([vp, vp], ctypes.c_int),
        "flb_batch_retire": ([vp, vp], ctypes.c_int),
        "flb_batch_step": ([vp, i64], ctypes.c_int),
        "flb_batch_size": ([vp, ctypes.POINTER(i32)], ctypes.c_int),
        "flb_batch_sync": ([vp], ctypes.c_int),
        "flb_batch_destroy": ([vp], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def check(rc):
    if rc < 0:
        raise FlbError(rc, load().flb_last_error().decode())
    return rc


def _ptr(a):
    """Data pointer of a numpy array or a torch tensor."""
    if isinstance(a, np.ndarray):
        return a.ctypes.data_as(ctypes.c_void_p)
    return ctypes.c_void_p(a.data_ptr())


def constants(model, theta=0.0):
    """The library's weights w (Q,) and moment basis m (Q, Q)."""
    lib = load()
    d = MODELS[model]
    Q = 2 * d + 1
    w = np.zeros(Q)
    m = np.zeros((Q, Q))
    check(lib.flb_lattice_constants(d, float(theta), _ptr(w), _ptr(m)))
    return w, m


def make_params(model, dims, precision=4, theta=0.0, omega=1.0, omega_n=0.0, omega_s=0.0,
                seed=0, noise="local", law="gauss", kernel="auto", tile_x=0, tile_rows=0, nt_store=0,
                pipeline=0, layout="two"):
    d = MODELS[model]
    dims = tuple(int(x) for x in dims) + (1,) * (3 - len(dims))
    p = Params()
    p.model = d
    p.precision = int(precision)
    for a in range(3):
        p.n[a] = dims[a]
    p.theta = float(theta)
    p.omega[0], p.omega[1], p.omega[2] = float(omega), float(omega_n), float(omega_s)
    p.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    p.noise = NOISE[noise]
    p.noise_law = LAWS[law]
    p.layout = LAYOUTS[layout]
    p.kernel = KERNELS[kernel]
    p.tile_x = int(tile_x)
    p.tile_rows = int(tile_rows)
    p.nt_store = int(nt_store)
    p.pipeline = int(pipeline)
    return p


def required_bytes(p):
    pop = ctypes.c_size_t()
    work = ctypes.c_size_t()
    check(load().flb_required_bytes(ctypes.byref(p), ctypes.byref(pop), ctypes.byref(work)))
    return pop.value, work.value


def _torch():
    import torch
    return torch


class Lattice:
    """One periodic lattice on a GPU.  Populations and workspace are torch
    uint8 device tensors owned by this object; the stream defaults to the
    device's current torch stream."""

    def __init__(self, model, dims, precision=4, device=None, stream=None, **kw):
        torch = _torch()
        lib = load()
        self.d = MODELS[model]
        self.Q = 2 * self.d + 1
        self.dims = tuple(int(x) for x in dims)
        if len(self.dims) != self.d:
            raise ValueError(f"a {self.d}-D model needs {self.d} sizes")
        self.precision = int(precision)
        self.dtype = np.float32 if self.precision == 4 else np.float64
        self.params = make_params(self.d, self.dims, precision, **kw)
        pop_bytes, work_bytes = required_bytes(self.params)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        with torch.cuda.device(self.device):
            self._pop = torch.empty(pop_bytes + 256, dtype=torch.uint8, device=self.device)
            self._work = torch.empty(work_bytes + 256, dtype=torch.uint8, device=self.device)
            pop_ptr = (self._pop.data_ptr() + 255) // 256 * 256
            work_ptr = (self._work.data_ptr() + 255) // 256 * 256
            h = ctypes.c_void_p()
            check(lib.flb_create(ctypes.byref(self.params), ctypes.c_void_p(pop_ptr), pop_bytes,
                                 ctypes.c_void_p(work_ptr), work_bytes,
                                 ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self.handle = h
        self.pop_bytes, self.work_bytes = pop_bytes, work_bytes
        self.shape = (self.Q,) + tuple(reversed(self.dims))
        self.nsite = int(np.prod(self.dims))

    # -- state -------------------------------------------------------------
    def set_populations(self, f, step=0):
        torch = _torch()
        if isinstance(f, np.ndarray):
            a = np.ascontiguousarray(f, dtype=self.dtype)
            if a.shape != self.shape:
                raise ValueError(f"expected shape {self.shape}, got {a.shape}")
            check(load().flb_set_populations(self.handle, _ptr(a), 0, int(step)))
        else:
            t = f.contiguous()
            if tuple(t.shape) != self.shape or t.element_size() != self.precision:
                raise ValueError("tensor shape or dtype does not match the lattice")
            check(load().flb_set_populations(self.handle, _ptr(t), 1 if t.is_cuda else 0, int(step)))
            del torch

    def get_populations(self):
        out = np.empty(self.shape, dtype=self.dtype)
        check(load().flb_get_populations(self.handle, _ptr(out), 0))
        return out

    def get_populations_device(self, out):
        check(load().flb_get_populations(self.handle, _ptr(out), 1))
        return out

    def step(self, n=1):
        check(load().flb_step(self.handle, int(n)))

    def set_check(self, every):
        """Check mode: flb_step checks for non-finite populations every
        `every` steps and at the end of each call (FLB_ENONFINITE); 0 = off."""
        check(load().flb_set_check(self.handle, int(every)))

    @property
    def t(self):
        v = ctypes.c_int64()
        check(load().flb_get_step(self.handle, ctypes.byref(v)))
        return v.value

    def sync(self):
        check(load().flb_sync(self.handle))

    # -- statistics --------------------------------------------------------
    def moments(self):
        m = Moments()
        check(load().flb_moments(self.handle, ctypes.byref(m)))
        return self._moments_dict(m)

    def set_moment_sampling(self, every):
        """Accumulate the lattice sums on the device every `every` steps."""
        check(load().flb_set_moment_sampling(self.handle, int(every)))

    def sampled_moments(self):
        """(sums over the samples, number of samples)."""
        m = Moments()
        n = ctypes.c_int64()
        check(load().flb_sampled_moments(self.handle, ctypes.byref(m), ctypes.byref(n)))
        return self._moments_dict(m), n.value

    def set_correlation(self, every, kvecs=None, nlag=1):
        """Accumulate S_ij(k) and the density time correlator every `every`
        steps for the wave vectors `kvecs` (nk x d integers); every = 0 stops."""
        if every == 0:
            check(load().flb_set_correlation(self.handle, 0, None, 0, 0))
            return
        kv = self._kvec(kvecs)
        self._corr_shape = (len(kv), int(nlag))
        check(load().flb_set_correlation(self.handle, int(every), kv.ctypes.data, len(kv), int(nlag)))

    def correlation(self):
        """(S_ij sums (nk, Q, Q) complex, C sums (nk, nlag) complex, nsamples)."""
        n = ctypes.c_int64()
        if getattr(self, "_corr_shape", None) is None:   # the library reports the state error
            check(load().flb_correlation(self.handle, None, None, ctypes.byref(n)))
        nk, nlag = self._corr_shape
        sij = np.zeros((nk, self.Q, self.Q, 2))
        ct = np.zeros((nk, nlag, 2))
        check(load().flb_correlation(self.handle, sij.ctypes.data, ct.ctypes.data, ctypes.byref(n)))
        return sij[..., 0] + 1j * sij[..., 1], ct[..., 0] + 1j * ct[..., 1], n.value

    def fourier_amplitudes(self):
        """f_i(k) of the current state for the correlation k-list: (nk, Q) complex."""
        if getattr(self, "_corr_shape", None) is None:
            check(load().flb_fourier_amplitudes(self.handle, None))
        nk, _ = self._corr_shape
        a = np.zeros((nk, self.Q, 2))
        check(load().flb_fourier_amplitudes(self.handle, a.ctypes.data))
        return a[..., 0] + 1j * a[..., 1]

    def set_regions(self, region=None, theta=(), omega=()):
        """Per-site region index (array of the lattice's shape, (.., y, x))
        with theta[r] and omega[r] = omega_j or (omega_j, omega_n, omega_s)
        per region; region=None returns to the uniform lattice."""
        if region is None:
            check(load().flb_set_regions(self.handle, None, 0, None, None))
            return
        reg = np.ascontiguousarray(region, dtype=np.uint8).reshape(-1)
        th = np.ascontiguousarray(theta, dtype=np.float64)
        om = np.zeros((len(th), 3))
        for r, o in enumerate(omega):
            o = np.atleast_1d(np.asarray(o, dtype=np.float64))
            om[r, :len(o)] = o
        check(load().flb_set_regions(self.handle, reg.ctypes.data, len(th), th.ctypes.data, om.ctypes.data))

    def profile(self, axis=0):
        """(sum of rho, sum of rho^2) over the sites of each coordinate along `axis`."""
        L = self.dims[axis]
        s, s2 = np.zeros(L), np.zeros(L)
        check(load().flb_profile(self.handle, int(axis), s.ctypes.data, s2.ctypes.data))
        return s, s2

    def profile_noalloc(self, axis, out_rho, out_rho2):
        """The density profile into caller device tensors (n[axis] doubles
        each), asynchronously, with no allocation (flb_profile_noalloc)."""
        check(load().flb_profile_noalloc(self.handle, int(axis), _ptr(out_rho), _ptr(out_rho2)))
        return out_rho, out_rho2

    def _moments_dict(self, m):
        Q = self.Q
        ff = np.zeros((Q, Q))
        k = 0
        for i in range(Q):
            for j in range(i, Q):
                ff[i, j] = ff[j, i] = m.sum_ff[k]
                k += 1
        return {
            "step": m.step, "nsite": m.nsite, "mass": m.mass, "mass0": m.mass0,
            "rho_eq": m.rho_eq, "sum_f": np.array(m.sum_f[:Q]), "sum_ff": ff,
            "sum_rho2": m.sum_rho2, "sum_rho_pos": m.sum_rho_pos,
            "n_negative": m.n_negative, "nonfinite": m.nonfinite,
        }

    def _kvec(self, kvecs):
        k = np.zeros((len(kvecs), 3), dtype=np.int32)
        kk = np.asarray(kvecs, dtype=np.int64).reshape(len(kvecs), -1 if len(kvecs) else 1)
        k[:, :kk.shape[1]] = kk
        return np.ascontiguousarray(k)

    def structure_factor(self, kvecs=None, mode="snapshot"):
        lib = load()
        modes = {"snapshot": SK_SNAPSHOT, "sample": SK_SAMPLE, "read": SK_READ, "reset": SK_RESET}
        md = modes[mode]
        if kvecs is None:
            kp, nk = None, 0
        else:
            kv = self._kvec(kvecs)
            kp, nk = _ptr(kv), len(kv)
        out = np.zeros(max(nk, 1024), dtype=np.float64)
        check(lib.flb_structure_factor(self.handle, kp, nk, md, _ptr(out)))
        if md == SK_RESET:
            self._sk_nk = nk
        if md == SK_SNAPSHOT:
            return out[:nk].copy()
        if md == SK_READ:  # the accumulator's k-list length when this object set it
            n = getattr(self, "_sk_nk", None)
            return out[:n].copy() if n is not None else out
        return None

    def set_sampling(self, every, kvecs=None):
        """Accumulate S(k) of kvecs while stepping, every `every` steps."""
        if every and kvecs is not None:
            kv = self._kvec(kvecs)
            check(load().flb_set_sampling(self.handle, int(every), _ptr(kv), len(kv)))
            self._sk_nk = len(kv)
        else:
            check(load().flb_set_sampling(self.handle, 0, None, 0))

    def close(self):
        if getattr(self, "handle", None):
            check(load().flb_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """A set of lattices advanced together (flb_batch_*): work-list launches
    (one workgroup per tile of a member) for lattices in HBM, one per step
    or per two-step pass, whole chunks of steps in LDS for small D1Q3
    lattices, chunks captured in a HIP graph.  Results are bit-identical to
    stepping each member alone."""

    def __init__(self, chunk=16, use_graph=True, lds_max_bytes=0, workers=0, item_rows=0, tiling=0,
                 stream=None, depth=0, width=0):
        o = BatchOpts()
        o.chunk, o.use_graph, o.lds_max_bytes, o.workers = int(chunk), int(bool(use_graph)), int(lds_max_bytes), int(workers)
        o.item_rows = int(item_rows)
        o.tiling = int(tiling)
        o.depth = int(depth)
        o.width = int(width)
        o.hip_stream = ctypes.c_void_p(stream.cuda_stream) if stream is not None else None
        h = ctypes.c_void_p()
        check(load().flb_batch_create(ctypes.byref(o), ctypes.byref(h)))
        self.handle = h
        self.members = []

    def admit(self, lat):
        check(load().flb_batch_admit(self.handle, lat.handle))
        self.members.append(lat)

    def retire(self, lat):
        check(load().flb_batch_retire(self.handle, lat.handle))
        self.members.remove(lat)

    def step(self, n=1):
        check(load().flb_batch_step(self.handle, int(n)))

    def sync(self):
        check(load().flb_batch_sync(self.handle))

    def __len__(self):
        v = ctypes.c_int32()
        check(load().flb_batch_size(self.handle, ctypes.byref(v)))
        return v.value

    def close(self):
        if getattr(self, "handle", None):
            check(load().flb_batch_destroy(self.handle))
            self.handle = None
            self.members = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def noise_sample(model, seed, step, site0, nsite, precision=8, law="gauss", device=None):
    """Philox words (nblock*4, nsite) uint32 and variates (Q-1, nsite) of the
    device noise stream."""
    torch = _torch()
    d = MODELS[model]
    Q = 2 * d + 1
    nblk = (Q - 1 + 3) // 4
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    words = torch.empty((nblk * 4, nsite), dtype=torch.int32, device=dev)
    vdt = torch.float32 if precision == 4 else torch.float64
    var = torch.empty((Q - 1, nsite), dtype=vdt, device=dev)
    st = torch.cuda.current_stream(dev)
    check(load().flb_noise_sample(d, precision, LAWS[law], int(seed) & 0xFFFFFFFFFFFFFFFF,
                                  int(step), int(site0), int(nsite), _ptr(words), _ptr(var),
                                  ctypes.c_void_p(st.cuda_stream)))
    st.synchronize()
    return words.cpu().numpy().view(np.uint32), var.cpu().numpy()


def gauss_map(r0, r1, precision=8, device=None):
    """The device Box-Muller map on Philox words r0, r1 (uint32 arrays of one
    length): returns (sqrt(-2 ln u0) cos 2 pi u1, sqrt(-2 ln u0) sin 2 pi u1)
    as the step kernels compute it."""
    torch = _torch()
    r0 = np.ascontiguousarray(r0, dtype=np.uint32)
    r1 = np.ascontiguousarray(r1, dtype=np.uint32)
    if r0.shape != r1.shape or r0.ndim != 1:
        raise ValueError("r0 and r1 must be 1-D arrays of one length")
    n = r0.size
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    words = torch.from_numpy(np.concatenate([r0, r1]).view(np.int32)).to(dev)
    z = torch.empty((2, n), dtype=torch.float32 if precision == 4 else torch.float64, device=dev)
    st = torch.cuda.current_stream(dev)
    check(load().flb_gauss_map(int(precision), _ptr(words), int(n), _ptr(z), ctypes.c_void_p(st.cuda_stream)))
    st.synchronize()
    out = z.cpu().numpy()
    return out[0], out[1]
