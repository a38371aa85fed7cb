"""ctypes wrapper around the FP64 C oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg.  The library path never imports this package.
Arrays are numpy, row-major ``[y, x]``; the C side is plain double precision.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# a prebuilt library to load instead (the pins' mutant test builds copies of
# oracle.c with one planted mistake each and runs the pins against them)
_LIB_OVERRIDE = os.environ.get("MPR_ORACLE_LIB")

OK, ERR_ARG, ERR_DEGENERATE = 0, 1, 2
MODE_FULL, MODE_OR_ONLY = 0, 1
FLAG_KEPT, FLAG_ACCEPTED, FLAG_WRAPPED, FLAG_UPDATED = 1, 2, 4, 8
INIT_SWEEP = 0xFFFFFFFF
TABLE_STREAM = 0x80000000


class Params(C.Structure):
    _fields_ = [
        ("q", C.c_double), ("R", C.c_int32), ("K", C.c_int32),
        ("n_f", C.c_int32), ("n_fit", C.c_int32), ("sg_degree", C.c_int32),
        ("a_targ", C.c_double), ("k_a", C.c_double), ("i_max", C.c_int32),
        ("fixed_relax", C.c_int32), ("eq_a_mode", C.c_int32), ("pad", C.c_int32),
        ("seed", C.c_uint64), ("stream", C.c_uint32), ("pad2", C.c_uint32),
    ]


class ChainStats(C.Structure):
    _fields_ = [
        ("relax_sweeps", C.c_int32), ("not_converged", C.c_int32),
        ("a_final", C.c_double), ("A_last", C.c_double), ("k_last", C.c_double),
    ]


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so (plain gcc, IEEE double)."""
    if (not force and os.path.exists(_LIB)
            and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC)):
        return _LIB
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared",
                           "-fno-fast-math", "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(_LIB_OVERRIDE if _LIB_OVERRIDE else build())
        _declare(_lib)
    return _lib


def _declare(L):
    d, i32, i64, u32, u64 = C.c_double, C.c_int, C.c_long, C.c_uint32, C.c_uint64
    P = C.c_void_p
    L.oracle_philox4x32_10.argtypes = [P, P, P]
    L.oracle_site_uniforms.argtypes = [u64, i32, i32, i32, u32, u32, u32, P, P]
    L.oracle_map_to_angles.argtypes = [i32, i32, P, P, P, P]
    L.oracle_map_to_angles.restype = i32
    L.oracle_energy.argtypes = [i32, i32, P, d]
    L.oracle_energy.restype = d
    L.oracle_bond_count.argtypes = [i32, i32]
    L.oracle_bond_count.restype = i64
    L.oracle_sample_energy.argtypes = [i32, i32, P, P, d, P, P]
    L.oracle_sample_energy.restype = i32
    L.oracle_half_sweep.argtypes = [i32, i32, P, P, i32, d, d, d, u64, u32, u32, u32, i32, P]
    L.oracle_half_sweep.restype = i64
    L.oracle_sg_slope.argtypes = [P, i32, i32]
    L.oracle_sg_slope.restype = d
    L.oracle_simulate.argtypes = [i32, i32, P, P, d, C.POINTER(Params), P, P, P, P,
                                  C.POINTER(ChainStats), P, i32, P, P, P]
    L.oracle_simulate.restype = i32
    L.oracle_predict.argtypes = [i32, i32, P, P, P, i32, P, P]
    L.oracle_spread.argtypes = [i32, i32, P, P, P, i32, P, P]
    L.oracle_quantiles.argtypes = [i32, i32, P, P, P, i32, P, i32, P, P]
    L.oracle_holdout_mask.argtypes = [i32, i32, P, u64, d, P]
    L.oracle_quantiles.restype = i32
    L.oracle_energy_table.argtypes = [i32, i32, d, i32, P, i32, i32, d, d, u64, u32, P]
    L.oracle_energy_table.restype = i32
    L.oracle_temperature_grid.argtypes = [i32, d, d, P]
    L.oracle_invert_temperature.argtypes = [i32, P, P, d, P, P]
    L.oracle_invert_temperature.restype = i32


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _u8(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.uint8)


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: status {code}")
        self.code = code


def default_params(**kw) -> Params:
    p = Params(q=0.5, R=1, K=10, n_f=5, n_fit=20, sg_degree=1, a_targ=0.3, k_a=3.0,
               i_max=20000, fixed_relax=-1, eq_a_mode=0, pad=0, seed=3000, stream=0, pad2=0)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


# ------------------------------------------------------------------ calls
def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def philox4x32_10_np(ctr, key) -> np.ndarray:
    """Philox4x32-10 (Salmon et al., SC'11) of many counters at once, in numpy:
    ctr (n, 4) uint32, key (2,) uint32 -> (n, 4) uint32.  A second, vectorised
    implementation beside the C one (each round: two 32 x 32 -> 64-bit
    products of counter words 0 and 2 with the round multipliers, their high
    halves xored with words 1, 3 and the key, the key bumped by the Weyl
    constants), for comparisons over millions of counters."""
    c = np.array(ctr, dtype=np.uint64).reshape(-1, 4)
    k0, k1 = np.uint64(int(key[0]) & 0xFFFFFFFF), np.uint64(int(key[1]) & 0xFFFFFFFF)
    m0, m1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
    w0, w1 = np.uint64(0x9E3779B9), np.uint64(0xBB67AE85)
    lo = np.uint64(0xFFFFFFFF)
    s32 = np.uint64(32)
    x0, x1, x2, x3 = c[:, 0], c[:, 1], c[:, 2], c[:, 3]
    for _ in range(10):
        p0 = m0 * x0
        p1 = m1 * x2
        x0, x1, x2, x3 = (p1 >> s32) ^ x1 ^ k0, p1 & lo, (p0 >> s32) ^ x3 ^ k1, p0 & lo
        k0 = (k0 + w0) & lo
        k1 = (k1 + w1) & lo
    return np.stack([x0, x1, x2, x3], axis=1).astype(np.uint32)


def site_uniforms(seed, nx, x, y, sweep, chain, stream):
    u, r = C.c_double(), C.c_double()
    lib().oracle_site_uniforms(seed, nx, x, y, sweep, chain, stream, C.byref(u), C.byref(r))
    return u.value, r.value


def map_to_angles(z, sampled):
    z, s = _f64(z), _u8(sampled)
    ny, nx = z.shape
    phi = np.zeros_like(z)
    zz = np.zeros(2)
    rc = lib().oracle_map_to_angles(nx, ny, _p(z), _p(s), _p(phi), _p(zz))
    if rc:
        raise OracleError(rc, "map_to_angles")
    return phi, zz


def energy(phi, q=0.5) -> float:
    phi = _f64(phi)
    ny, nx = phi.shape
    return lib().oracle_energy(nx, ny, _p(phi), q)


def bond_count(nx, ny) -> int:
    return lib().oracle_bond_count(nx, ny)


def sample_energy(phi, sampled, q=0.5):
    phi, s = _f64(phi), _u8(sampled)
    ny, nx = phi.shape
    e, n = C.c_double(), C.c_long()
    rc = lib().oracle_sample_energy(nx, ny, _p(phi), _p(s), q, C.byref(e), C.byref(n))
    if rc:
        raise OracleError(rc, "sample_energy")
    return e.value, n.value


def half_sweep(phi, sampled, colour, T, a, sweep, chain=0, stream=0, seed=3000, q=0.5,
               mode=MODE_FULL, with_flags=False):
    """One half-sweep in place on a float64 copy; returns (phi, accepted, flags)."""
    phi = _f64(phi).copy()
    s = _u8(sampled)
    ny, nx = phi.shape
    flags = np.zeros((ny, nx), dtype=np.uint8) if with_flags else None
    acc = lib().oracle_half_sweep(nx, ny, _p(phi), _p(s), colour, T, a, q, seed, sweep, chain,
                                  stream, mode, _p(flags) if with_flags else None)
    return phi, acc, flags


def sg_slope(e, degree=1) -> float:
    e = _f64(e)
    return lib().oracle_sg_slope(_p(e), e.size, degree)


def simulate(phi, sampled, T, params: Params, phi_init=None, trace_len=0, want_last=False, want_sq=False,
             want_states=False, want_control=False):
    """Returns (phi_sum, stats, e_trace, phi_last), then phi_sq_sum (sum of
    the squared states at gap sites) when want_sq, then the M = R K states
    (array M x ny x nx, state r K + k) when want_states, then (a_trace,
    acc_trace) when want_control: per chain and sweep t < trace_len
    (relaxation and equilibrium) the a its proposals used and the accepted
    count (NaN past the chain's last sweep)."""
    phi, s = _f64(phi), _u8(sampled)
    ny, nx = phi.shape
    phi_sum = np.zeros_like(phi)
    phi_sq = np.zeros_like(phi) if want_sq else None
    states = np.zeros((params.R * params.K,) + phi.shape) if want_states else None
    stats = (ChainStats * params.R)()
    trace = np.zeros((params.R, trace_len)) if trace_len else None
    last = np.zeros_like(phi) if want_last else None
    init = _f64(phi_init) if phi_init is not None else None
    a_tr = np.full((params.R, trace_len), np.nan) if want_control else None
    acc_tr = np.full((params.R, trace_len), np.nan) if want_control else None
    rc = lib().oracle_simulate(nx, ny, _p(phi), _p(s), T, C.byref(params),
                               _p(init) if init is not None else None, _p(phi_sum),
                               _p(phi_sq) if phi_sq is not None else None,
                               _p(states) if states is not None else None, stats,
                               _p(trace) if trace is not None else None, trace_len,
                               _p(last) if last is not None else None,
                               _p(a_tr) if a_tr is not None else None,
                               _p(acc_tr) if acc_tr is not None else None)
    if rc:
        raise OracleError(rc, "simulate")
    st = [dict(relax_sweeps=c.relax_sweeps, not_converged=c.not_converged, a_final=c.a_final,
               A_last=c.A_last, k_last=c.k_last) for c in stats]
    out = (phi_sum, st, trace, last)
    if want_sq:
        out += (phi_sq,)
    if want_states:
        out += (states,)
    if want_control:
        out += ((a_tr, acc_tr),)
    return out


def spread(sampled, phi_sum, phi_sq_sum, M, zmin_zmax):
    """Standard deviation over the M realizations of the back-transformed
    value at each gap site (0 at samples, and for M = 1)."""
    s, ps, pq = _u8(sampled), _f64(phi_sum), _f64(phi_sq_sum)
    ny, nx = ps.shape
    zz = _f64(zmin_zmax)
    out = np.zeros_like(ps)
    lib().oracle_spread(nx, ny, _p(s), _p(ps), _p(pq), M, _p(zz), _p(out))
    return out


def quantiles(z, sampled, states, probs, zmin_zmax):
    """Per-site quantiles (probs) of the back-transformed states (M x ny x nx);
    data values at sampled sites.  Returns an array len(probs) x ny x nx."""
    z, s = _f64(z), _u8(sampled)
    st = _f64(states)
    pr = _f64(probs)
    ny, nx = z.shape
    out = np.zeros((pr.size, ny, nx))
    zz = _f64(zmin_zmax)
    rc = lib().oracle_quantiles(nx, ny, _p(z), _p(s), _p(st), st.shape[0], _p(pr), pr.size, _p(zz), _p(out))
    if rc:
        raise OracleError(rc, "quantiles")
    return out


def holdout_mask(sampled, seed, hold):
    """1 at the samples kept for fitting, 0 at gaps and held-out samples."""
    s = _u8(sampled)
    ny, nx = s.shape
    fit = np.zeros_like(s)
    lib().oracle_holdout_mask(nx, ny, _p(s), seed, hold, _p(fit))
    return fit


def select_q(z, sampled, params: Params, q_grid, holdout, nT, T_lo, T_hi, burn, meas):
    """The hold-out choice of q (the paper gives no rule): hide the samples
    of holdout_mask, and for each candidate q estimate T from the rest
    (sample energy and the e(T, L) table with that q), simulate, predict the
    hidden samples and take their mean absolute error; the smallest wins (on
    a tie, the larger q).  Returns (q_best, errors, temperatures)."""
    z = _f64(z)
    s = _u8(sampled)
    ny, nx = z.shape
    fit = holdout_mask(s, params.seed, holdout)
    hidden = (s == 1) & (fit == 0)
    phi, zz = map_to_angles(z, fit)
    Tg = temperature_grid(nT, T_lo, T_hi)
    errs, temps = [], []
    for q in q_grid:
        e_s, _ = sample_energy(phi, fit, q)
        et = energy_table(nx, ny, Tg, burn, meas, a_targ=params.a_targ, k_a=params.k_a, seed=params.seed, q=q)
        T, _ = invert_temperature(Tg, et, e_s)
        p = Params.from_buffer_copy(params)
        p.q = q
        ps, _, _, _ = simulate(phi, fit, T, p)
        zh = predict(z, fit, ps, p.R * p.K, zz)
        errs.append(float(np.mean(np.abs(z[hidden] - zh[hidden]))))
        temps.append(T)
    best = 0
    for k in range(1, len(q_grid)):
        if errs[k] < errs[best] or (errs[k] == errs[best] and q_grid[k] > q_grid[best]):
            best = k
    return q_grid[best], np.array(errs), np.array(temps)


def predict(z, sampled, phi_sum, M, zmin_zmax):
    z, s, ps = _f64(z), _u8(sampled), _f64(phi_sum)
    ny, nx = z.shape
    zz = _f64(zmin_zmax)
    out = np.zeros_like(z)
    lib().oracle_predict(nx, ny, _p(z), _p(s), _p(ps), M, _p(zz), _p(out))
    return out


def temperature_grid(nT, T_lo, T_hi) -> np.ndarray:
    out = np.zeros(nT)
    lib().oracle_temperature_grid(nT, T_lo, T_hi, _p(out))
    return out


def energy_table(nx, ny, Tg, n_burn, n_meas, a_targ=0.3, k_a=3.0, seed=3000,
                 stream=TABLE_STREAM, q=0.5) -> np.ndarray:
    Tg = _f64(Tg)
    out = np.zeros(Tg.size)
    rc = lib().oracle_energy_table(nx, ny, q, Tg.size, _p(Tg), n_burn, n_meas, a_targ, k_a,
                                   seed, stream, _p(out))
    if rc:
        raise OracleError(rc, "energy_table")
    return out


def invert_temperature(Tg, e, e_s):
    Tg, e = _f64(Tg), _f64(e)
    T, cl = C.c_double(), C.c_int()
    rc = lib().oracle_invert_temperature(Tg.size, _p(Tg), _p(e), e_s, C.byref(T), C.byref(cl))
    if rc:
        raise OracleError(rc, "invert_temperature")
    return T.value, bool(cl.value)
