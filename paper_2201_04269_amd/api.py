"""Python API over libmbc: index sets, plans, contract, backward, autograd.

PyTorch provides device memory and the current stream only; every step of the
correlator evaluation runs in libmbc's HIP kernels.
"""
import ctypes

import numpy as np
import torch

from . import _binding as B


def _op_descs(ops):
    arr = (B.OpDesc * len(ops))()
    for i, od in enumerate(ops):
        arr[i].op = B.OPS[od["op"]]
        arr[i].snk_spin = int(od.get("snk_spin", 0))
        arr[i].src_spin = int(od.get("src_spin", od.get("snk_spin", 0)))
        arr[i].sign_mode = B.SIGNS[od.get("sign_mode", "exact")]
        arr[i].symmetrise = 1 if od.get("symmetrise", True) else 0
    return arr


class IndexSet:
    """Index set I and exact weights of a batch of correlators (host, integer).

    ``ops``: list of dicts with keys op ("proton", "neutron", "DI", "DII",
    "HE3_I", "HE3_II"), snk_spin, src_spin, sign_mode ("exact"/"r2"),
    symmetrise (bool).  Mirrors mbc_build_index_set.
    """

    def __init__(self, ops):
        self.ops = [dict(o) for o in ops]
        h = ctypes.c_void_p()
        descs = _op_descs(self.ops)
        B.check(B.lib().mbc_build_index_set(descs, len(self.ops), ctypes.byref(h)))
        self._h = h
        self._free = B.lib().mbc_index_set_free
        nu, nd, nc = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        nnz = ctypes.c_int64()
        B.check(B.lib().mbc_index_set_dims(h, ctypes.byref(nu), ctypes.byref(nd), ctypes.byref(nnz),
                                           ctypes.byref(nc)))
        self.n_u, self.n_d, self.nnz, self.n_corr = nu.value, nd.value, nnz.value, nc.value
        self._export = None

    def export(self):
        """dict of numpy arrays: snk_u, src_u, snk_d, src_d, corr_id, w_re, w_im, w_den."""
        if self._export is None:
            n, nu, nd = self.nnz, self.n_u, self.n_d
            out = dict(snk_u=np.zeros((n, nu), np.int32), src_u=np.zeros((n, nu), np.int32),
                       snk_d=np.zeros((n, nd), np.int32), src_d=np.zeros((n, nd), np.int32),
                       corr_id=np.zeros(n, np.int32), w_re=np.zeros(n, np.int64),
                       w_im=np.zeros(n, np.int64), w_den=np.zeros(self.n_corr, np.int64))
            ptr = [out[k].ctypes.data_as(ctypes.c_void_p) for k in
                   ("snk_u", "src_u", "snk_d", "src_d", "corr_id", "w_re", "w_im", "w_den")]
            B.check(B.lib().mbc_index_set_export(self._h, *ptr))
            self._export = out
        return self._export

    def weights(self):
        """Exact weights as complex128 (num / den)."""
        e = self.export()
        den = e["w_den"][e["corr_id"]].astype(float)
        return (e["w_re"].astype(float) + 1j * e["w_im"].astype(float)) / den

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._free(h)
            self._h = None


def _stream_ptr(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Plan:
    """Compiled evaluation schedule of an index set, resident on the device."""

    def __init__(self, iset, precision="f64", stream=None):
        self.iset = iset
        self.precision = precision
        prec = {"f64": B.F64, "f32c": B.F32C}[precision]
        h = ctypes.c_void_p()
        B.check(B.lib().mbc_plan_create(iset._h, prec, _stream_ptr(stream), ctypes.byref(h)))
        self._h = h
        self._free = B.lib().mbc_plan_destroy
        st = B.PlanStats()
        B.check(B.lib().mbc_plan_get_stats(h, ctypes.byref(st)))
        self.stats = {k: getattr(st, k) for k, _ in B.PlanStats._fields_}

    @property
    def n_corr(self):
        return self.iset.n_corr

    def workspace_bytes(self, T, V, backward=False):
        n = ctypes.c_size_t()
        B.check(B.lib().mbc_plan_workspace_bytes(self._h, int(T), int(V), 1 if backward else 0,
                                                 ctypes.byref(n)))
        return n.value

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._free(h)
            self._h = None


def _check_S(S_u, S_d):
    for S in (S_u, S_d):
        if not (S.is_cuda and S.is_contiguous() and S.dim() == 4 and S.shape[-2:] == (12, 12)):
            raise ValueError("S must be a contiguous CUDA tensor [T, V, 12, 12]")
        if S.dtype not in (torch.complex128, torch.complex64):
            raise ValueError("S must be complex128 or complex64")
    if S_u.shape != S_d.shape or S_u.dtype != S_d.dtype:
        raise ValueError("S_u and S_d must have the same shape and dtype")
    return B.C128 if S_u.dtype == torch.complex128 else B.C64


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def contract(plan, S_u, S_d, W=None, stream=None):
    """C[c, t] (complex128 [n_corr, T]) of eq. 1 for propagators [T, V, 12, 12]."""
    dt = _check_S(S_u, S_d)
    T, V = S_u.shape[:2]
    if W is not None:
        if W.dtype != torch.complex128 or not W.is_cuda or W.numel() != plan.iset.nnz:
            raise ValueError("W must be a CUDA complex128 tensor of nnz entries")
        W = W.contiguous()
    C = torch.empty((plan.n_corr, T), dtype=torch.complex128, device=S_u.device)
    nbytes = plan.workspace_bytes(T, V)
    ws = torch.empty(max(nbytes, 16), dtype=torch.uint8, device=S_u.device)
    B.check(B.lib().mbc_contract(plan._h, _ptr(S_u), _ptr(S_d), dt, int(T), int(V), _ptr(W), _ptr(C),
                                 _ptr(ws), ctypes.c_size_t(ws.numel()), _stream_ptr(stream)))
    return C


def contract_noalloc(plan, S_u, S_d, C, W=None, stream=None):
    """mbc_contract_noalloc: eq. 1 into the caller's C (complex128 [n_corr, T])
    with the library's fixed per-GPU scratch instead of a workspace; nothing
    is allocated by this call.  Overlapping calls on one GPU race."""
    dt = _check_S(S_u, S_d)
    T, V = S_u.shape[:2]
    if W is not None and (W.dtype != torch.complex128 or not W.is_cuda or W.numel() != plan.iset.nnz
                          or not W.is_contiguous()):
        raise ValueError("W must be a contiguous CUDA complex128 tensor of nnz entries")
    if C.dtype != torch.complex128 or not C.is_cuda or tuple(C.shape) != (plan.n_corr, T) or not C.is_contiguous():
        raise ValueError("C must be a contiguous CUDA complex128 tensor [n_corr, T]")
    B.check(B.lib().mbc_contract_noalloc(plan._h, _ptr(S_u), _ptr(S_d), dt, int(T), int(V), _ptr(W), _ptr(C),
                                         _stream_ptr(stream)))
    return C


def contract_backward(plan, S_u, S_d, W, grad_C, need_W=True, need_S=True, stream=None):
    """(grad_W, grad_S_u, grad_S_d) of mbc_contract_backward (None where not requested)."""
    dt = _check_S(S_u, S_d)
    T, V = S_u.shape[:2]
    grad_C = grad_C.to(torch.complex128).contiguous()
    gW = torch.empty(plan.iset.nnz, dtype=torch.complex128, device=S_u.device) if need_W else None
    gSu = torch.empty_like(S_u) if need_S else None
    gSd = torch.empty_like(S_d) if need_S else None
    nbytes = plan.workspace_bytes(T, V, backward=True)
    ws = torch.empty(max(nbytes, 16), dtype=torch.uint8, device=S_u.device)
    if W is not None:
        W = W.contiguous()
    B.check(B.lib().mbc_contract_backward(plan._h, _ptr(S_u), _ptr(S_d), dt, int(T), int(V), _ptr(W),
                                          _ptr(grad_C), _ptr(gW), _ptr(gSu), _ptr(gSd), _ptr(ws),
                                          ctypes.c_size_t(ws.numel()), _stream_ptr(stream)))
    return gW, gSu, gSd


class Contract(torch.autograd.Function):
    """C = Contract.apply(S_u, S_d, W, plan): differentiable in S_u, S_d and W.

    The backward is libmbc's adjoint kernels (Jacobi's formula through the
    Laplace recursion for dS, per-entry site sums for dW), with every minor
    recomputed rather than stored.
    """

    @staticmethod
    def forward(ctx, S_u, S_d, W, plan):
        ctx.plan = plan
        ctx.save_for_backward(S_u, S_d, W)
        return contract(plan, S_u, S_d, W)

    @staticmethod
    def backward(ctx, grad_C):
        S_u, S_d, W = ctx.saved_tensors
        need_S = ctx.needs_input_grad[0] or ctx.needs_input_grad[1]
        need_W = ctx.needs_input_grad[2]
        gW, gSu, gSd = contract_backward(ctx.plan, S_u, S_d, W, grad_C, need_W=need_W, need_S=need_S)
        return (gSu if ctx.needs_input_grad[0] else None,
                gSd if ctx.needs_input_grad[1] else None,
                gW if need_W else None, None)


# ---------------------------------------------------------------------------
# Hadron blocks and block-level correlators (include/mbc_blocks.h)
# ---------------------------------------------------------------------------
def _block_descs(corrs):
    arr = (B.BlockCorrDesc * len(corrs))()
    for i, c in enumerate(corrs):
        arr[i].op = B.OPS[c["op"]]
        arr[i].snk_spin = int(c.get("snk_spin", 0))
        arr[i].src_spin = int(c.get("src_spin", c.get("snk_spin", 0)))
        arr[i].sign_mode = B.SIGNS[c.get("sign_mode", "exact")]
        for s, mom in enumerate(c.get("moms", [])):
            for d in range(3):
                arr[i].mom[s][d] = int(mom[d])
        for s, pt in enumerate(c.get("src_pts", [])):
            arr[i].src_pt[s] = int(pt)
    return arr


class BlockSet:
    """Block types and merged product terms of block-level correlators (host).

    ``corrs``: list of dicts with keys op, snk_spin, src_spin, sign_mode,
    moms (one integer momentum triple per baryon slot, written order) and
    optionally src_pts (the source point, 0..2, of each source baryon slot;
    default all 0, a local source).  Mirrors mbc_block_set_build.
    """

    def __init__(self, corrs):
        self.corrs = [dict(c) for c in corrs]
        h = ctypes.c_void_p()
        B.check(B.lib().mbc_block_set_build(_block_descs(self.corrs), len(self.corrs), ctypes.byref(h)))
        self._h = h
        self._free = B.lib().mbc_block_set_free
        nc, ns, nt, npt = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        nterms = ctypes.c_int64()
        B.check(B.lib().mbc_block_set_dims(h, ctypes.byref(nc), ctypes.byref(ns), ctypes.byref(nt),
                                           ctypes.byref(nterms), ctypes.byref(npt)))
        self.n_corr, self.n_slots, self.n_types, self.n_terms = nc.value, ns.value, nt.value, nterms.value
        self.n_points = npt.value

    def types(self, with_points=False):
        """List of (family "p"/"n", projector, momentum triple) in block order,
        each with the source points of its antiquarks (A, Y, C) appended when
        ``with_points``."""
        fam = np.zeros(self.n_types, np.int32)
        proj = np.zeros(self.n_types, np.int32)
        mom = np.zeros((self.n_types, 3), np.int32)
        src = np.zeros((self.n_types, 3), np.int32)
        B.check(B.lib().mbc_block_set_types(self._h, fam.ctypes.data_as(ctypes.c_void_p),
                                            proj.ctypes.data_as(ctypes.c_void_p),
                                            mom.ctypes.data_as(ctypes.c_void_p),
                                            src.ctypes.data_as(ctypes.c_void_p)))
        out = []
        for f, p, m, z in zip(fam, proj, mom, src):
            rec = (B.FAMILIES[int(f)], int(p), tuple(int(v) for v in m))
            out.append(rec + (tuple(int(v) for v in z),) if with_points else rec)
        return out

    def export(self):
        """dict of numpy arrays: factor [n_terms, n_slots], corr_id, num_re, num_im, den."""
        n = self.n_terms
        out = dict(factor=np.zeros((n, self.n_slots), np.int32), corr_id=np.zeros(n, np.int32),
                   num_re=np.zeros(n, np.int64), num_im=np.zeros(n, np.int64),
                   den=np.zeros(self.n_corr, np.int64))
        ptr = [out[k].ctypes.data_as(ctypes.c_void_p) for k in ("factor", "corr_id", "num_re", "num_im", "den")]
        B.check(B.lib().mbc_block_set_export(self._h, *ptr))
        return out

    def factor_tree(self, corr):
        """(factors, children) of correlator ``corr``'s linearised factor tree;
        its leaves are the correlator's terms in export order."""
        n = ctypes.c_int64()
        B.check(B.lib().mbc_block_set_factor_tree(self._h, int(corr), ctypes.byref(n), None, None))
        fac = np.zeros(n.value, np.int32)
        ch = np.zeros(n.value, np.int32)
        B.check(B.lib().mbc_block_set_factor_tree(self._h, int(corr), ctypes.byref(n),
                                                  fac.ctypes.data_as(ctypes.c_void_p),
                                                  ch.ctypes.data_as(ctypes.c_void_p)))
        return fac, ch

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._free(h)
            self._h = None


def block_multiplicities(corr, max_terms=1 << 26):
    """(n_terms, n_distinct, hist) of mbc_block_multiplicities for one correlator dict."""
    d = _block_descs([corr])
    nt, nd, mm = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    B.check(B.lib().mbc_block_multiplicities(d, int(max_terms), ctypes.byref(nt), ctypes.byref(nd),
                                             ctypes.byref(mm), None, 0))
    hist = np.zeros(mm.value + 1, np.int64)
    B.check(B.lib().mbc_block_multiplicities(d, int(max_terms), ctypes.byref(nt), ctypes.byref(nd),
                                             ctypes.byref(mm), hist.ctypes.data_as(ctypes.c_void_p),
                                             hist.shape[0]))
    return nt.value, nd.value, hist


class BlockPlan:
    """A block set's types and terms, resident on the device."""

    def __init__(self, bset, stream=None):
        self.bset = bset
        h = ctypes.c_void_p()
        B.check(B.lib().mbc_block_plan_create(bset._h, _stream_ptr(stream), ctypes.byref(h)))
        self._h = h
        self._free = B.lib().mbc_block_plan_destroy
        st = B.BlockPlanStats()
        B.check(B.lib().mbc_block_plan_get_stats(h, ctypes.byref(st)))
        self.stats = {k: getattr(st, k) for k, _ in B.BlockPlanStats._fields_}

    def workspace_bytes(self, T, dims):
        n = ctypes.c_size_t()
        d = (ctypes.c_int32 * 3)(*[int(v) for v in dims])
        B.check(B.lib().mbc_block_workspace_bytes(self._h, int(T), d, ctypes.byref(n)))
        return n.value

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._free(h)
            self._h = None


def _workspace(plan, T, dims, device):
    return torch.empty(max(plan.workspace_bytes(T, dims), 16), dtype=torch.uint8, device=device)


def blocks(plan, S_u, S_d, dims, workspace=None, stream=None):
    """Momentum-projected blocks [T, n_types, 4, 12, 12, 12] complex128 (mbc_blocks_compute).

    S_u, S_d: [T, V, 12, 12], or [n_points, T, V, 12, 12] with one set per
    source point."""
    npts = plan.bset.n_points
    if S_u.dim() == 5 and S_d.dim() == 5:
        if S_u.shape[0] != npts or S_d.shape[0] != npts:
            raise ValueError(f"propagators must hold {npts} source-point sets")
        dt = _check_S(S_u[0], S_d[0])
        if not (S_u.is_contiguous() and S_d.is_contiguous()):
            raise ValueError("S must be contiguous")
        T, V = S_u.shape[1:3]
    else:
        if npts != 1:
            raise ValueError(f"the block set uses {npts} source points: pass [n_points, T, V, 12, 12]")
        dt = _check_S(S_u, S_d)
        T, V = S_u.shape[:2]
    if V != dims[0] * dims[1] * dims[2]:
        raise ValueError("sites per timeslice must equal L1 L2 L3")
    out = torch.empty((T, plan.bset.n_types, 4, 12, 12, 12), dtype=torch.complex128, device=S_u.device)
    ws = workspace if workspace is not None else _workspace(plan, T, dims, S_u.device)
    d = (ctypes.c_int32 * 3)(*[int(v) for v in dims])
    B.check(B.lib().mbc_blocks_compute(plan._h, _ptr(S_u), _ptr(S_d), dt, int(T), d, _ptr(out), _ptr(ws),
                                       ctypes.c_size_t(ws.numel()), _stream_ptr(stream)))
    return out


def block_contract(plan, blk, method="tree", workspace=None, stream=None):
    """C [n_corr, T] complex128 from blocks (mbc_block_contract); method
    "tree" (linearised factor trees) or "terms" (one product per term)."""
    if not (blk.is_cuda and blk.dtype == torch.complex128 and blk.is_contiguous()):
        raise ValueError("blocks must be a contiguous CUDA complex128 tensor")
    T = blk.shape[0]
    C = torch.empty((plan.bset.n_corr, T), dtype=torch.complex128, device=blk.device)
    ws = workspace if workspace is not None else _workspace(plan, T, (1, 1, 1), blk.device)
    B.check(B.lib().mbc_block_contract(plan._h, _ptr(blk), int(T), B.BLOCK_METHODS[method], _ptr(C), _ptr(ws),
                                       ctypes.c_size_t(ws.numel()), _stream_ptr(stream)))
    return C


def block_correlators(plan, S_u, S_d, dims, method="tree", stream=None):
    """(C [n_corr, T], blocks): the blocks of every type, then their contraction."""
    blk = blocks(plan, S_u, S_d, dims, stream=stream)
    return block_contract(plan, blk, method=method, stream=stream), blk


# ----------------------------------------------------------------------------
# Tensor e-graphs (mbc_egraph.h)
# ----------------------------------------------------------------------------
class TensorEGraph:
    """E-graph of a sum of tensor products and its extracted plan (Sec. 5).

    tensors: list of (extents, symmetries) with symmetries a list of
    (slot permutation, sign); terms: list of (coef, [(tensor, labels)]).
    Use ``TensorEGraph.for_blocks`` for a block-level correlator.  objective:
    "flops" (smallest tree cost, the default) or "reuse" (the paper's)."""

    def __init__(self, tensors=None, terms=None, node_limit=100000, objective="flops", _handle=None):
        L = B.lib()
        if _handle is None:
            decl = (B.TensorDecl * len(tensors))()
            for i, (ext, syms) in enumerate(tensors):
                decl[i].rank = len(ext)
                for k, e in enumerate(ext):
                    decl[i].ext[k] = int(e)
                decl[i].n_sym = len(syms)
                for g, (perm, sign) in enumerate(syms):
                    for k, p in enumerate(perm):
                        decl[i].perm[g][k] = int(p)
                    decl[i].sign[g] = int(sign)
            nf = sum(len(f) for _, f in terms)
            fac = (B.TensorFactor * max(nf, 1))()
            begin = np.zeros(len(terms) + 1, dtype=np.int32)
            coef = np.zeros((len(terms), 2))
            q = 0
            for k, (c, factors) in enumerate(terms):
                coef[k] = (complex(c).real, complex(c).imag)
                for t, labels in factors:
                    fac[q].tensor = int(t)
                    for s, x in enumerate(labels):
                        fac[q].label[s] = int(x)
                    q += 1
                begin[k + 1] = q
            h = ctypes.c_void_p()
            B.check(L.mbc_egraph_build(decl, len(tensors), fac, begin.ctypes.data_as(ctypes.c_void_p),
                                       coef.ctypes.data_as(ctypes.c_void_p), len(terms), int(node_limit),
                                       B.EXTRACT[objective], ctypes.byref(h)))
            _handle = h
        self._h = _handle
        self._free = L.mbc_egraph_free
        st = B.EGraphStats()
        B.check(L.mbc_egraph_get_stats(self._h, ctypes.byref(st)))
        self.stats = {k: getattr(st, k) for k, _ in B.EGraphStats._fields_ if k != "out_ext"}
        self.out_shape = tuple(st.out_ext[k] for k in range(st.n_open))

    @classmethod
    def for_blocks(cls, bset, corr=0, node_limit=100000, objective="flops"):
        """The block-level correlator `corr` of a BlockSet (mbc_egraph_build_blocks)."""
        h = ctypes.c_void_p()
        B.check(B.lib().mbc_egraph_build_blocks(bset._h, int(corr), int(node_limit), B.EXTRACT[objective],
                                                ctypes.byref(h)))
        g = cls(_handle=h)
        g.n_block_types = bset.n_types
        return g

    def export(self):
        """Parsed mbc_egraph_export: classes, terms (with coefficients) and plan steps."""
        L = B.lib()
        n = ctypes.c_int64()
        B.check(L.mbc_egraph_export(self._h, None, 0, ctypes.byref(n)))
        buf = np.zeros(n.value, dtype=np.int32)
        B.check(L.mbc_egraph_export(self._h, buf.ctypes.data_as(ctypes.c_void_p), n.value, ctypes.byref(n)))
        v = buf.tolist()
        p = 0

        def take(k):
            nonlocal p
            out = v[p:p + k]
            p += k
            return out

        classes = []
        for _ in range(take(1)[0]):
            rep, nf, no, lc = take(4)
            code = tuple(take(lc))
            nodes = []
            for _ in range(take(1)[0]):
                c1, c2, sign, n1 = take(4)
                o1 = tuple(take(n1))
                o2 = tuple(take(take(1)[0]))
                nodes.append((c1, c2, sign, o1, o2))
            classes.append(dict(rep=rep, n_factors=nf, n_open=no, code=code, nodes=nodes))
        terms = []
        for _ in range(take(1)[0]):
            c, no = take(2)
            terms.append((c, tuple(take(no))))
        steps = [tuple(take(2)) for _ in range(take(1)[0])]
        coef = np.zeros((len(terms), 2))
        if terms:
            B.check(L.mbc_egraph_term_coefs(self._h, coef.ctypes.data_as(ctypes.c_void_p)))
        return dict(classes=classes, terms=terms, coefs=coef[:, 0] + 1j * coef[:, 1], steps=steps)

    def workspace_bytes(self, batch=1):
        n = ctypes.c_size_t()
        B.check(B.lib().mbc_egraph_workspace_bytes(self._h, int(batch), ctypes.byref(n)))
        return n.value

    def execute(self, inputs, batch=1, batch_strides=None, stream=None):
        """[batch, *out_shape] complex128: inputs is a list (one per tensor id) of
        CUDA complex128 tensors, or None for a library constant; batch_strides
        in complex elements (default: 0, shared)."""
        nt = self.stats["n_tensors"]
        if len(inputs) != nt:
            raise ValueError(f"{nt} inputs expected")
        dev = next(t.device for t in inputs if t is not None)
        for t in inputs:
            if t is not None and not (t.is_cuda and t.dtype == torch.complex128 and t.is_contiguous()):
                raise ValueError("inputs must be contiguous CUDA complex128 tensors")
        ptrs = (ctypes.c_void_p * nt)(*[t.data_ptr() if t is not None else 0 for t in inputs])
        bs = np.zeros(nt, dtype=np.int64) if batch_strides is None else np.asarray(batch_strides, dtype=np.int64)
        out = torch.empty((int(batch),) + self.out_shape, dtype=torch.complex128, device=dev)
        ws = torch.empty(max(self.workspace_bytes(batch), 16), dtype=torch.uint8, device=dev)
        B.check(B.lib().mbc_egraph_execute(self._h, ptrs, bs.ctypes.data_as(ctypes.c_void_p), int(batch), _ptr(out),
                                           _ptr(ws), ctypes.c_size_t(ws.numel()), _stream_ptr(stream)))
        return out

    def execute_blocks(self, blk, workspace=None, stream=None):
        """C[t] (complex128 [T]) of a for_blocks graph from blocks [T, n_types, 4, 12, 12, 12]."""
        T, nty = blk.shape[0], blk.shape[1]
        if nty != self.n_block_types:
            raise ValueError("blocks of another block set")
        flat = blk.reshape(T, nty, 6912)
        inputs = [flat[0, y] for y in range(nty)] + [None] * (self.stats["n_tensors"] - nty)
        strides = [nty * 6912] * nty + [0] * (self.stats["n_tensors"] - nty)
        # inputs[y] views the first timeslice of type y; entry t is t * n_types * 6912 further on
        return self._execute_views(inputs, blk, T, strides, workspace, stream)

    def _execute_views(self, inputs, base, batch, strides, workspace, stream):
        nt = self.stats["n_tensors"]
        ptrs = (ctypes.c_void_p * nt)(*[t.data_ptr() if t is not None else 0 for t in inputs])
        bs = np.asarray(strides, dtype=np.int64)
        out = torch.empty((int(batch),) + self.out_shape, dtype=torch.complex128, device=base.device)
        ws = workspace
        if ws is None:
            ws = torch.empty(max(self.workspace_bytes(batch), 16), dtype=torch.uint8, device=base.device)
        B.check(B.lib().mbc_egraph_execute(self._h, ptrs, bs.ctypes.data_as(ctypes.c_void_p), int(batch), _ptr(out),
                                           _ptr(ws), ctypes.c_size_t(ws.numel()), _stream_ptr(stream)))
        return out

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._free(h)
            self._h = None


# ----------------------------------------------------------------------------
# Linearised factor trees over arbitrary factor sets (mbc_tree.h)
# ----------------------------------------------------------------------------
class FactorTree:
    """A linearised factor tree (Sec. 4): the paper's factors / children /
    coefficients arrays in depth-first order (factors[0] = -1, the root),
    factors indexing a table of n_values factor values."""

    def __init__(self, factors, children, coefficients, n_values, stream=None):
        L = B.lib()
        f = np.ascontiguousarray(factors, dtype=np.int32)
        ch = np.ascontiguousarray(children, dtype=np.int32)
        c = np.asarray(coefficients, dtype=np.complex128).reshape(-1)
        coef = np.ascontiguousarray(np.stack([c.real, c.imag], axis=-1).reshape(-1))
        if f.shape != ch.shape:
            raise ValueError("factors and children must have one entry per vertex")
        h = ctypes.c_void_p()
        B.check(L.mbc_factor_tree_create(f.ctypes.data_as(ctypes.c_void_p), ch.ctypes.data_as(ctypes.c_void_p),
                                         f.shape[0], coef.ctypes.data_as(ctypes.c_void_p), c.shape[0],
                                         int(n_values), _stream_ptr(stream), ctypes.byref(h)))
        self._h = h
        self._free = L.mbc_factor_tree_destroy
        self.n_values = int(n_values)
        d, fl = ctypes.c_int32(), ctypes.c_double()
        B.check(L.mbc_factor_tree_stats(h, ctypes.byref(d), ctypes.byref(fl)))
        self.depth, self.flops = d.value, fl.value

    def evaluate(self, values, stream=None):
        """[batch] complex128: the tree's value for each row of values
        ([batch, n_values] CUDA complex128)."""
        if not (values.is_cuda and values.dtype == torch.complex128 and values.is_contiguous()
                and values.dim() == 2 and values.shape[1] == self.n_values):
            raise ValueError(f"values must be a contiguous CUDA complex128 tensor [batch, {self.n_values}]")
        batch = values.shape[0]
        out = torch.empty(batch, dtype=torch.complex128, device=values.device)
        n = ctypes.c_size_t()
        B.check(B.lib().mbc_factor_tree_workspace_bytes(self._h, batch, ctypes.byref(n)))
        ws = torch.empty(max(n.value, 16), dtype=torch.uint8, device=values.device)
        B.check(B.lib().mbc_factor_tree_evaluate(self._h, _ptr(values), batch, _ptr(out), _ptr(ws),
                                                 ctypes.c_size_t(ws.numel()), _stream_ptr(stream)))
        return out

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._free(h)
            self._h = None
