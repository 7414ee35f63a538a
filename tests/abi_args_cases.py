"""Argument-error paths of every C-ABI entry point, checked on a context
without a device (oica_create with OICA_NO_DEVICE), so they run on a host with
no GPU.  Each call must return its documented code; a call whose arguments are
valid must stop with OICA_E_DEVICE where device work would begin.  The
pointers passed as "valid" are never dereferenced on the host (the calls stop
before any device work), so a fixed non-null address stands in for them.

Run as a script (``python tests/abi_args_cases.py LIB``) it checks the library
at LIB and exits non-zero on a mismatch: the sanitizer test runs it that way
under AddressSanitizer / UndefinedBehaviorSanitizer.
"""
import ctypes as C
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

OK, E_ARG, E_SHAPE, E_RANK, E_NONFINITE, E_DEVICE, E_NOMEM, E_UNSUP, E_NOCONV = \
    0, -1, -2, -3, -4, -5, -6, -7, -8
F64, F32, BF16 = 0, 1, 2


def open_lib(path):
    from paper_2408_17118_amd import oica
    lib = C.CDLL(path)
    for name, (res, args) in oica._SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


def run(lib):
    """Returns the list of mismatches (empty when every path answers as documented)."""
    from paper_2408_17118_amd import oica
    bad = []
    P = C.c_void_p(0x10000)            # stands in for a valid device or host pointer
    NUL = None
    ctx = C.c_void_p()
    assert lib.oica_create(C.byref(ctx), -1, NUL) == OK and ctx.value
    assert lib.oica_create(NUL, 0, NUL) == E_ARG

    def expect(label, got, want):
        if got != want:
            bad.append(f"{label}: got {got}, want {want} "
                       f"({lib.oica_last_error(ctx).decode(errors='replace')})")

    def fp(**kw):
        d = dict(max_iter=100, tol=1e-6, precision=F32, tol_bf16=1e-5, refine_iters=5, traj_iters=0,
                 check_every=4, profile=0, refine_groups=1, pruner=None, prune_pass=0,
                 guard_top=0, guard_min=0)
        d.update(kw)
        return oica.FpParams(**d)

    # ---- whitening
    def wh(N=8, T=100, X=P, raw=F64, ld=100, Xw=P, out=F32):
        return lib.oica_whiten(ctx, N, T, X, raw, ld, Xw, out, NUL, NUL, NUL, NUL)
    expect("whiten N=0", wh(N=0), E_ARG)
    expect("whiten N>max", wh(N=129), E_UNSUP)
    expect("whiten T<=N", wh(T=8, ld=8), E_ARG)
    expect("whiten T huge", wh(T=(1 << 40) + 1, ld=(1 << 40) + 1), E_UNSUP)
    expect("whiten X null", wh(X=NUL), E_ARG)
    expect("whiten Xw null", wh(Xw=NUL), E_ARG)
    expect("whiten raw bf16", wh(raw=BF16), E_UNSUP)
    expect("whiten ld<T", wh(ld=99), E_SHAPE)
    expect("whiten out f64", wh(out=F64), E_UNSUP)
    expect("whiten valid", wh(), E_DEVICE)
    expect("whiten null ctx", lib.oica_whiten(NUL, 8, 100, P, F64, 100, P, F32, NUL, NUL, NUL, NUL), E_ARG)

    # ---- batched whitening
    arr = (oica.WhitenProblem * 2)()
    for d in range(2):
        arr[d] = oica.WhitenProblem(8, 100, P, F64, 100, P, NUL, NUL, NUL, NUL, 0)
    expect("whiten_batched D=0", lib.oica_whiten_batched(ctx, 0, arr, F32), E_ARG)
    expect("whiten_batched D>1024", lib.oica_whiten_batched(ctx, 1025, arr, F32), E_ARG)
    expect("whiten_batched null", lib.oica_whiten_batched(ctx, 2, NUL, F32), E_ARG)
    expect("whiten_batched out", lib.oica_whiten_batched(ctx, 2, arr, F64), E_UNSUP)
    arr[1].ld_raw = 50
    expect("whiten_batched ld", lib.oica_whiten_batched(ctx, 2, arr, F32), E_SHAPE)
    arr[1].ld_raw = 100
    arr[1].X_raw = NUL
    expect("whiten_batched X null", lib.oica_whiten_batched(ctx, 2, arr, F32), E_ARG)
    arr[1].X_raw = P
    arr[1].N = 0
    expect("whiten_batched N", lib.oica_whiten_batched(ctx, 2, arr, F32), E_ARG)
    arr[1].N = 8
    expect("whiten_batched valid", lib.oica_whiten_batched(ctx, 2, arr, F32), E_DEVICE)

    # ---- fixed point
    def fpc(N=8, T=100, Xw=P, xt=F32, X32=P, K=16, W0=P, p=None, W=P, traj=NUL):
        prm = p if p is not None else fp()
        return lib.oica_fixed_point(ctx, N, T, Xw, xt, X32, K, W0, C.byref(prm), W, P, P, P, traj, NUL)
    expect("fp K=0", fpc(K=0), E_ARG)
    expect("fp K huge", fpc(K=(1 << 24) + 1), E_UNSUP)
    expect("fp N=0", fpc(N=0), E_ARG)
    expect("fp max_iter", fpc(p=fp(max_iter=0)), E_ARG)
    expect("fp tol", fpc(p=fp(tol=0.0)), E_ARG)
    expect("fp tol nan", fpc(p=fp(tol=float("nan"))), E_ARG)
    expect("fp precision", fpc(p=fp(precision=F64)), E_UNSUP)
    expect("fp tol_bf16", fpc(xt=BF16, p=fp(precision=BF16, tol_bf16=-1.0)), E_ARG)
    expect("fp refine", fpc(p=fp(refine_iters=-1)), E_ARG)
    expect("fp traj", fpc(p=fp(traj_iters=17)), E_ARG)
    expect("fp traj null", fpc(p=fp(traj_iters=4)), E_ARG)
    expect("fp check_every", fpc(p=fp(check_every=-1)), E_ARG)
    expect("fp row terms", fpc(p=fp(bf16_row_terms=5)), E_ARG)
    expect("fp row terms neg", fpc(p=fp(bf16_row_terms=-1)), E_ARG)
    expect("fp switch step", fpc(p=fp(bf16_switch_step=-1.0)), E_ARG)
    expect("fp switch step inf", fpc(p=fp(bf16_switch_step=float("inf"))), E_ARG)
    expect("fp Xw null", fpc(Xw=NUL), E_ARG)
    expect("fp W0 null", fpc(W0=NUL), E_ARG)
    expect("fp bf16 dtype", fpc(xt=F32, p=fp(precision=BF16)), E_ARG)
    expect("fp f32 dtype", fpc(xt=BF16), E_ARG)
    expect("fp params null", lib.oica_fixed_point(ctx, 8, 100, P, F32, P, 16, P, NUL, P, P, P, P,
                                                   NUL, NUL), E_ARG)
    expect("fp valid", fpc(), E_DEVICE)
    expect("fp valid bf16", fpc(xt=BF16, p=fp(precision=BF16)), E_DEVICE)

    # ---- batched fixed point
    pr = (oica.Problem * 2)()
    for d in range(2):
        pr[d] = oica.Problem(8, 1000, 64, P, P, P, P, P, P, P)
    bp = oica.BatchParams(0, NUL, 0, 0)
    st = oica.BatchStats()

    def fpb(D=2, xt=F32, p=None):
        prm = p if p is not None else fp()
        return lib.oica_fixed_point_batched(ctx, D, pr, xt, C.byref(prm), C.byref(bp), C.byref(st))
    expect("fpb D=0", fpb(D=0), E_ARG)
    expect("fpb traj", fpb(p=fp(traj_iters=2)), E_ARG)
    expect("fpb dtype", fpb(xt=BF16), E_ARG)
    pr[1].K = 0
    expect("fpb K", fpb(), E_ARG)
    pr[1].K = 64
    pr[1].W0 = NUL
    expect("fpb null", fpb(), E_ARG)
    pr[1].W0 = P
    pr[1].N = 200
    expect("fpb N", fpb(), E_UNSUP)
    pr[1].N = 8
    expect("fpb valid", fpb(), E_DEVICE)

    # ---- one update, kurtosis
    expect("update dtype", lib.oica_update(ctx, 8, 100, P, F64, 16, P, P, P), E_UNSUP)
    expect("update K", lib.oica_update(ctx, 8, 100, P, F32, 0, P, P, P), E_ARG)
    expect("update null", lib.oica_update(ctx, 8, 100, P, F32, 16, NUL, P, P), E_ARG)
    expect("update valid", lib.oica_update(ctx, 8, 100, P, F32, 16, P, P, P), E_DEVICE)
    expect("kurtosis K", lib.oica_kurtosis(ctx, 8, 100, P, 0, P, P), E_ARG)
    expect("kurtosis null", lib.oica_kurtosis(ctx, 8, 100, NUL, 4, P, P), E_ARG)
    expect("kurtosis valid", lib.oica_kurtosis(ctx, 8, 100, P, 4, P, P), E_DEVICE)
    expect("kurtosis_noalloc K", lib.oica_kurtosis_noalloc(ctx, 8, 100, P, 0, P, P), E_ARG)
    expect("kurtosis_noalloc big", lib.oica_kurtosis_noalloc(ctx, 1, 4, P, 2_200_000, P, P), E_UNSUP)
    expect("kurtosis_noalloc valid", lib.oica_kurtosis_noalloc(ctx, 8, 100, P, 4, P, P), E_DEVICE)

    # ---- unique
    nu, na = C.c_int(0), C.c_int(0)

    def un(K=16, tau=1e-3, n_top=0, cap=4, U=P, W=P):
        prm = oica.UniqueParams(tau, 1, n_top)
        return lib.oica_unique(ctx, 8, 100, K, W, P, P, C.byref(prm), cap, U, P, P, P, P, NUL,
                               C.byref(nu), C.byref(na))
    expect("unique K", un(K=0), E_ARG)
    expect("unique tau 0", un(tau=0.0), E_ARG)
    expect("unique tau 1", un(tau=1.0), E_ARG)
    expect("unique n_top", un(n_top=-1), E_ARG)
    expect("unique cap", un(cap=-1), E_ARG)
    expect("unique W null", un(W=NUL), E_ARG)
    expect("unique U null", un(U=NUL), E_ARG)
    expect("unique valid", un(), E_DEVICE)
    expect("unique cap 0", un(cap=0, U=NUL), E_DEVICE)
    up = (oica.UniqueProblem * 1)()
    up[0] = oica.UniqueProblem(8, 100, 16, P, P, P, 4, P, P, P, P, P, NUL, 0, 0)
    prm = oica.UniqueParams(1e-3, 1, 0)
    expect("unique_batched D", lib.oica_unique_batched(ctx, 0, up, C.byref(prm)), E_ARG)
    expect("unique_batched valid", lib.oica_unique_batched(ctx, 1, up, C.byref(prm)), E_DEVICE)

    # ---- deflation driver
    nf = C.c_int(0)
    steps = (oica.DeflationStep * 8)()

    def dfl(N=8, L=16, tau=1e-3, p=None, W0=P, Wout=P):
        prm = p if p is not None else fp()
        return lib.oica_deflation(ctx, N, 100, P, L, W0, C.byref(prm), tau, 1, Wout, C.byref(nf), steps)
    expect("deflation L", dfl(L=0), E_ARG)
    expect("deflation tau", dfl(tau=1.5), E_ARG)
    expect("deflation traj", dfl(p=fp(traj_iters=2)), E_ARG)
    expect("deflation W0", dfl(W0=NUL), E_ARG)
    expect("deflation N", dfl(N=0), E_ARG)
    expect("deflation valid", dfl(), E_DEVICE)

    # ---- original algorithm
    def org(N=8, L=16, p=None, W0=P):
        prm = p if p is not None else fp()
        return lib.oica_ordering_original(ctx, N, 100, P, L, W0, C.byref(prm), 1e-3, 1, P,
                                          C.byref(nf), steps)
    expect("original L", org(L=0), E_ARG)
    expect("original bf16", org(p=fp(precision=BF16)), E_UNSUP)
    expect("original W0", org(W0=NUL), E_ARG)
    expect("original valid", org(), E_DEVICE)

    # ---- pruner (no pruner object can exist without a device)
    w = (C.c_float * oica.Pruner.N_PARAMS)()
    m16 = (C.c_float * 16)(*([0.0] * 16))
    s16 = (C.c_float * 16)(*([1.0] * 16))
    pr_out = C.c_void_p()
    expect("pruner_create null", lib.oica_pruner_create(ctx, NUL, m16, s16, C.byref(pr_out)), E_ARG)
    s16[3] = 0.0
    expect("pruner_create std", lib.oica_pruner_create(ctx, w, m16, s16, C.byref(pr_out)), E_ARG)
    s16[3] = 1.0
    expect("pruner_create valid", lib.oica_pruner_create(ctx, w, m16, s16, C.byref(pr_out)), E_DEVICE)
    expect("pruner_predict null", lib.oica_pruner_predict(ctx, NUL, P, 4, P), E_ARG)
    expect("pruner_set_threshold", lib.oica_pruner_set_threshold(NUL, 0.5), E_ARG)

    # ---- options, status strings
    expect("set_option unknown", lib.oica_set_option(99, 0), E_ARG)
    expect("set_option sweeps", lib.oica_set_option(2, 31), E_ARG)
    expect("set_option give-up", lib.oica_set_option(1, 2), E_ARG)
    v = C.c_int(-1)
    expect("get_option sweeps", lib.oica_get_option(2, C.byref(v)), OK)
    if v.value != 30:
        bad.append(f"default sweep limit {v.value}")
    expect("get_option null", lib.oica_get_option(2, NUL), E_ARG)
    for code in (OK, E_ARG, E_SHAPE, E_RANK, E_NONFINITE, E_DEVICE, E_NOMEM, E_UNSUP, E_NOCONV, 123):
        if not lib.oica_status_string(code):
            bad.append(f"status string {code}")
    expect("set_stream null", lib.oica_set_stream(NUL, NUL), E_ARG)
    lib.oica_destroy(ctx)
    lib.oica_destroy(NUL)
    return bad


if __name__ == "__main__":
    lib = open_lib(sys.argv[1])
    mismatches = run(lib)
    for m in mismatches:
        print("MISMATCH", m)
    print(f"{len(mismatches)} mismatches")
    sys.exit(1 if mismatches else 0)
