"""ctypes binding of libspeedygs.so (declared in include/speedygs.h).

Argument marshalling only: every step of the RD path runs in the library's
HIP kernels.  Device buffers are passed as raw pointers (``tensor.data_ptr()``
of torch CUDA tensors); the stream is torch's current HIP stream.  Loading
fails loudly when the library is missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libspeedygs.so")

NCH = 59
STATS_WORDS = 128
RATE_GRAD_FLOATS = 256
SPLAT_FIELDS = 12

SGS_OK, SGS_EINVAL, SGS_ENOMEM, SGS_EHIP, SGS_ESTATE, SGS_ECAPACITY = 0, -1, -2, -3, -4, -5
_STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ESTATE", -5: "ECAPACITY"}


class SgsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class sgs_camera(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("fx", C.c_float),
                ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float),
                ("campos", C.c_float * 3)]


class sgs_options(C.Structure):
    _fields_ = [("tile_w", C.c_int32), ("tile_h", C.c_int32), ("tau", C.c_float),
                ("schedule", C.c_int32), ("deterministic", C.c_int32),
                ("reserved", C.c_int32 * 3)]


class sgs_rate_options(C.Structure):
    _fields_ = [("proxy", C.c_int32), ("masking", C.c_int32), ("alpha", C.c_float),
                ("reserved", C.c_int32)]


class sgs_adam_options(C.Structure):
    _fields_ = [("lr", C.c_float * 59), ("lr_q", C.c_float), ("lr_score", C.c_float),
                ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("sh_rest", C.c_int32), ("sparse", C.c_int32), ("reserved", C.c_int32),
                ("step", C.c_int64)]


class sgs_octree_header(C.Structure):
    _fields_ = [("depth", C.c_int64), ("kmin", C.c_int64 * 3), ("kept", C.c_int64),
                ("unique", C.c_int64), ("tokens", C.c_int64), ("dups", C.c_int64),
                ("flags", C.c_int64), ("level_size", C.c_int64 * 21)]


class sgs_fl_channel(C.Structure):
    _fields_ = [("q", C.c_float), ("kmin", C.c_int32), ("width", C.c_int32)]


class sgs_ans_stream(C.Structure):
    _fields_ = [("words", C.c_void_p), ("n_words", C.c_int64), ("block_off", C.c_void_p),
                ("n", C.c_int64), ("freq", C.c_void_p), ("sym", C.c_void_p),
                ("order", C.c_int32), ("lane_len", C.c_int32)]


OCTREE_HEADER_WORDS = C.sizeof(sgs_octree_header) // 8
assert OCTREE_HEADER_WORDS == 30

SCHEDULES = {"tile": 0, "stride": 1, "queue": 2, "block": 3}


P = C.c_void_p
I64 = C.c_int64
I32 = C.c_int32
U64 = C.c_uint64
F32 = C.c_float

_SIGS = {
    "sgs_create": [C.POINTER(P), C.c_int, P],
    "sgs_destroy": [P],
    "sgs_last_error": [P],
    "sgs_set_stream": [P, P],
    "sgs_set_scene": [P, I64, I64, I64, P, I32, I32, I32, P],
    "sgs_fakequant_prune": [P, P, P, P, I32, P, U64, U64, P, P, P, P],
    "sgs_rate_proxy": [P, P, P, F32, P, P],
    "sgs_render_fwd": [P, P, P, P, P, P, P],
    "sgs_l1_loss": [P, P, P, F32, P, P],
    "sgs_render_bwd": [P, P, P, P, P, P, P, P],
    "sgs_fakequant_prune_bwd": [P, P, P, P, I32, P, P, P, P, P, P, P],
    "sgs_quant_render_fwd": [P, P, P, P, I32, P, U64, U64, P, P, P, P, P, P, P],
    "sgs_quant_render_bwd": [P, P, P, P, I32, P, P, P, P, P, P, P, P, P],
    "sgs_query": [P, P, C.POINTER(I64), C.POINTER(U64)],
    "sgs_set_eval_count_mode": [P, I32],
    "sgs_set_grad_sh_rest": [P, I32],
    "sgs_query_items": [P, C.POINTER(I64)],
    "sgs_autotune": [P, P, P, P, P, I32, P, P],
    "sgs_copy_structure": [P, P, P, I64, P, P, P, P],
    "sgs_copy_splat_grads": [P, P],
    "sgs_profile_enable": [P, I32],
    "sgs_profile_read": [P, P, P],
    "sgs_reserve_pairs": [P, I64],
    "sgs_graph_begin": [P],
    "sgs_graph_end": [P, C.POINTER(P)],
    "sgs_graph_launch": [P, P],
    "sgs_graph_destroy": [P],
    "sgs_rate_mlp_pack": [P, P, P],
    "sgs_rate_mlp_fwd": [P, P, P, P, P, P, P, P, P],
    "sgs_rate_mlp_bwd": [P, P, P, P, P, P, P, P, I32, F32, P, P, P, P],
    "sgs_rate_mlp_infer": [P, P, P, P, I64, P],
    "sgs_rate_mlp_train_scratch_bytes": [I64],
    "sgs_rate_mlp_train_step": [P, P, P, P, P, P, P, I64, F32, I64, P, P, P],
    "sgs_rate_mlp_train_step_static": [P, P, P, P, P, P, P, I64, F32, I64, P, P],
    "sgs_adam_step": [P, P, P, P, P, P, P, P, P, P, P, P, P, P],
    "sgs_rate_mlp_features": [P, P, P, P, P, I64, P],
    "sgs_ssim_loss": [P, P, P, F32, P, P],
    "sgs_rate_variant": [P, P, P, P, P, F32, P, P],
    "sgs_rate_variant_bwd": [P, P, P],
    "sgs_compact": [P, P, I32, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.POINTER(I32),
                    I64, C.POINTER(I64)],
    "sgs_fl_encode": [P, P, P, P, P, P, I64, P],
    "sgs_fl_decode": [P, P, P, I64, I64, I64, P],
    "sgs_octree_encode": [P, P, I64, I64, P, P, P, I64, P, P, P, I64, P],
    "sgs_octree_decode": [P, P, P, P, P, P, P, P, I64, P],
    "sgs_ans_max_words": [I64, I32],
    "sgs_ans_model": [P, P, I64, I32, I32, P, P],
    "sgs_ans_encode": [P, P, I64, I32, I32, P, P, I64, P, P],
    "sgs_ans_decode": [P, P, I64, P, I64, I32, I32, P, P, P],
    "sgs_ans_decode_multi": [P, I32, P, P],
    "sgs_morton_order": [P, P, I64, I64, P, P, P, P, P],
    "sgs_attr_plane_rows": [P, P],
    "sgs_attr_planes": [P, P, I64, P, I64, P, P, I32, P],
    "sgs_attr_reconstruct": [P, P, I64, P, P, I32, P, I64],
    "sgs_positional_embedding": [P, P, I64, I64, I32, I32, P, P, P],
}
PROF_GROUPS = ("fakequant", "rate", "preprocess", "depth_sort", "scan", "duplicate",
               "tile_sort", "ranges", "blend_fwd", "l1", "grad_clear", "blend_bwd",
               "preprocess_bwd", "fakequant_bwd", "mlp_fwd", "mlp_bwd", "mlp_train", "codec",
               "adam", "ssim", "octree", "ans")
MLP_PARAMS = 24961
MLP_PACKED_BYTES = 98304
MLP_STATIC_ROWS = 8192
EXPORTS = tuple(_SIGS)

_lib = None


def lib(path: str | None = None):
    """Load libspeedygs.so (no compute call is made)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"libspeedygs.so not built ({p}); run __graft_entry__.build()")
    L = C.CDLL(p)
    for name, args in _SIGS.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = {"sgs_last_error": C.c_char_p, "sgs_destroy": None, "sgs_graph_destroy": None,
                     "sgs_rate_mlp_train_scratch_bytes": C.c_int64,
                     "sgs_ans_max_words": C.c_int64,
                     "sgs_attr_plane_rows": C.c_int64}.get(name, C.c_int)
    if path is None:
        _lib = L
    return L


def _ptr(x) -> int | None:
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def cameras(cams: np.ndarray):
    cams = np.ascontiguousarray(cams, np.float32)
    arr = (sgs_camera * cams.shape[0])()
    C.memmove(arr, cams.ctypes.data, cams.nbytes)
    return arr


class Graph:
    """An instantiated HIP graph of captured library calls."""

    def __init__(self, L, h):
        self.L, self.h = L, h

    def launch(self, stream):
        st = self.L.sgs_graph_launch(self.h, P(stream.cuda_stream))
        if st != SGS_OK:
            raise SgsError(st, "graph launch failed")

    def close(self):
        if self.h:
            self.L.sgs_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    """One library context bound to a device and torch's current stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self._torch = torch
        self.L = lib()
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        h = P()
        self._check(self.L.sgs_create(C.byref(h), device, P(stream.cuda_stream)), None)
        self.h = h

    def _check(self, st: int, h=None):
        if st != SGS_OK:
            msg = self.L.sgs_last_error(h if h is not None else getattr(self, "h", None))
            raise SgsError(st, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "h", None):
            self.L.sgs_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        self._check(self.L.sgs_set_stream(self.h, P(stream.cuda_stream)), self.h)

    # ---- the C ABI, one method per entry point -----------------------------
    def set_scene(self, n, npad, n_hat, cams, width, height, tile=(16, 16), tau=1.0,
                  schedule="tile", deterministic=False):
        """schedule: blend launch, one wave per 8x8 sub-tile: "tile" (one
        workgroup per sub-tile), "stride" or "queue" (resident workgroups over
        the sub-tiles of the tiles ordered by list length), "block" (resident
        workgroups of one whole tile each, striding over that order)."""
        cams = np.ascontiguousarray(cams, np.float32)
        arr = cameras(cams)
        opt = sgs_options(tile[0], tile[1], tau, SCHEDULES[schedule], int(bool(deterministic)),
                          (C.c_int32 * 3)())
        self.V, self.W, self.H, self.n, self.npad = cams.shape[0], width, height, n, npad
        self.tile = tile
        self.schedule = schedule
        self._check(self.L.sgs_set_scene(self.h, n, npad, n_hat, arr, cams.shape[0], width,
                                         height, C.byref(opt)), self.h)

    def fakequant_prune(self, params, qstep, score, mask_mode, given_mask, seed, step,
                        qparams, hard_mask, soft_mask, stats):
        self._check(self.L.sgs_fakequant_prune(
            self.h, _ptr(params), _ptr(qstep), _ptr(score), mask_mode, _ptr(given_mask),
            seed, step, _ptr(qparams), _ptr(hard_mask), _ptr(soft_mask), _ptr(stats)), self.h)

    def rate_proxy(self, stats, qstep, rate_weight, out3, rate_grad=None):
        self._check(self.L.sgs_rate_proxy(self.h, _ptr(stats), _ptr(qstep), rate_weight,
                                          _ptr(out3), _ptr(rate_grad)), self.h)

    def render_fwd(self, qparams, hard_mask, image, final_T, last, eval_count=None):
        self._check(self.L.sgs_render_fwd(self.h, _ptr(qparams), _ptr(hard_mask), _ptr(image),
                                          _ptr(final_T), _ptr(last), _ptr(eval_count)), self.h)

    def l1_loss(self, image, target, loss, dL_dimage, scale=1.0):
        self._check(self.L.sgs_l1_loss(self.h, _ptr(image), _ptr(target), scale, _ptr(loss),
                                       _ptr(dL_dimage)), self.h)

    def render_bwd(self, qparams, hard_mask, final_T, last, dL_dimage, grad_qparams,
                   grad_hard_mask):
        self._check(self.L.sgs_render_bwd(self.h, _ptr(qparams), _ptr(hard_mask), _ptr(final_T),
                                          _ptr(last), _ptr(dL_dimage), _ptr(grad_qparams),
                                          _ptr(grad_hard_mask)), self.h)

    def fakequant_prune_bwd(self, params, qstep, soft_mask, mask_mode, rate_grad, stats,
                            grad_qparams, grad_hard_mask, grad_params, grad_qstep, grad_score):
        self._check(self.L.sgs_fakequant_prune_bwd(
            self.h, _ptr(params), _ptr(qstep), _ptr(soft_mask), mask_mode, _ptr(rate_grad),
            _ptr(stats), _ptr(grad_qparams), _ptr(grad_hard_mask), _ptr(grad_params),
            _ptr(grad_qstep), _ptr(grad_score)), self.h)

    def quant_render_fwd(self, params, qstep, score, mask_mode, given_mask, seed, step,
                         hard_mask, soft_mask, stats, image, final_T, last, eval_count=None):
        """fakequant_prune + render_fwd without materializing the quantized rows."""
        self._check(self.L.sgs_quant_render_fwd(
            self.h, _ptr(params), _ptr(qstep), _ptr(score), mask_mode, _ptr(given_mask), seed,
            step, _ptr(hard_mask), _ptr(soft_mask), _ptr(stats), _ptr(image), _ptr(final_T),
            _ptr(last), _ptr(eval_count)), self.h)

    def quant_render_bwd(self, params, qstep, soft_mask, mask_mode, rate_grad, stats, final_T,
                         last, dL_dimage, grad_params, grad_qstep, grad_score, grad_hard_mask):
        """render_bwd + fakequant_prune_bwd over the raw rows."""
        self._check(self.L.sgs_quant_render_bwd(
            self.h, _ptr(params), _ptr(qstep), _ptr(soft_mask), mask_mode, _ptr(rate_grad),
            _ptr(stats), _ptr(final_T), _ptr(last), _ptr(dL_dimage), _ptr(grad_params),
            _ptr(grad_qstep), _ptr(grad_score), _ptr(grad_hard_mask)), self.h)

    def autotune(self, params, qstep, given_mask, target, reps: int = 3):
        """sgs_autotune: returns ((tile_w, tile_h), schedule name, [ms per
        candidate in the order timed]); the context stays bound with the choice."""
        opt = sgs_options()
        ms = (C.c_float * 8)()
        self._check(self.L.sgs_autotune(self.h, _ptr(params), _ptr(qstep), _ptr(given_mask),
                                        _ptr(target), int(reps), C.byref(opt), ms), self.h)
        names = {v: k for k, v in SCHEDULES.items()}
        self.tile = (opt.tile_w, opt.tile_h)
        self.schedule = names[opt.schedule]
        return self.tile, self.schedule, [float(v) for v in ms]

    def query_items(self) -> int:
        """(splat, super-tile) items of the last render (synchronizes)."""
        v = C.c_int64(0)
        self._check(self.L.sgs_query_items(self.h, C.byref(v)), self.h)
        return int(v.value)

    def set_eval_count_mode(self, mode: int):
        """0: the method's in-span evaluations (default); 1: the evaluations
        the timed blend performs after its reach test."""
        self._check(self.L.sgs_set_eval_count_mode(self.h, int(mode)), self.h)

    def set_grad_sh_rest(self, on: bool):
        """Whether the fused and learned-rate backward passes write the
        higher-SH gradient rows (channels 6-50) of grad_params."""
        self._check(self.L.sgs_set_grad_sh_rest(self.h, 1 if on else 0), self.h)

    def query(self, stats=None):
        pairs = I64()
        flags = U64()
        st = self.L.sgs_query(self.h, _ptr(stats), C.byref(pairs), C.byref(flags))
        self._check(st, self.h)
        return int(pairs.value), int(flags.value)

    def copy_structure(self, tile_ids=None, vals=None, cap=0, ranges=None, spans=None,
                       depth=None, splats=None):
        self._check(self.L.sgs_copy_structure(self.h, _ptr(tile_ids), _ptr(vals), cap,
                                              _ptr(ranges), _ptr(spans), _ptr(depth),
                                              _ptr(splats)), self.h)

    def copy_splat_grads(self, out):
        self._check(self.L.sgs_copy_splat_grads(self.h, _ptr(out)), self.h)

    # ---- device-side pair count and graph capture ----------------------------
    def reserve_pairs(self, capacity: int):
        self._check(self.L.sgs_reserve_pairs(self.h, capacity), self.h)

    def graph_begin(self):
        self._check(self.L.sgs_graph_begin(self.h), self.h)

    def graph_end(self) -> "Graph":
        g = P()
        self._check(self.L.sgs_graph_end(self.h, C.byref(g)), self.h)
        return Graph(self.L, g)

    # ---- learned rate estimator --------------------------------------------
    def rate_mlp_pack(self, theta, packed):
        self._check(self.L.sgs_rate_mlp_pack(self.h, _ptr(theta), _ptr(packed)), self.h)

    def rate_mlp_fwd(self, packed, theta, params, qstep, stats, hard_mask, out_R,
                     per_gaussian=None):
        self._check(self.L.sgs_rate_mlp_fwd(self.h, _ptr(packed), _ptr(theta), _ptr(params),
                                            _ptr(qstep), _ptr(stats), _ptr(hard_mask),
                                            _ptr(out_R), _ptr(per_gaussian)), self.h)

    def rate_mlp_bwd(self, packed, theta, params, qstep, stats, hard_mask, soft_mask, mask_mode,
                     rate_weight, grad_params, grad_qstep, grad_score=None, grad_hard_mask=None):
        self._check(self.L.sgs_rate_mlp_bwd(
            self.h, _ptr(packed), _ptr(theta), _ptr(params), _ptr(qstep), _ptr(stats),
            _ptr(hard_mask), _ptr(soft_mask), mask_mode, rate_weight, _ptr(grad_params),
            _ptr(grad_qstep), _ptr(grad_score), _ptr(grad_hard_mask)), self.h)

    def adam_step(self, lr, step, params, params_m, params_v, grad_params, q=None, q_m=None,
                  q_v=None, grad_q=None, score=None, s_m=None, s_v=None, grad_score=None,
                  lr_q=0.0, lr_score=0.0, beta1=0.9, beta2=0.999, eps=1e-8, sh_rest=True,
                  sparse=False):
        """One Adam step; lr: 59 per-channel learning rates (or one float)."""
        o = sgs_adam_options()
        lrs = [float(lr)] * 59 if isinstance(lr, (int, float)) else [float(a) for a in lr]
        if len(lrs) != 59:
            raise ValueError("lr needs 59 entries")
        o.lr = (C.c_float * 59)(*lrs)
        o.lr_q, o.lr_score = lr_q, lr_score
        o.beta1, o.beta2, o.eps = beta1, beta2, eps
        o.sh_rest, o.sparse, o.reserved, o.step = int(bool(sh_rest)), int(bool(sparse)), 0, step
        self._check(self.L.sgs_adam_step(
            self.h, C.byref(o), _ptr(params), _ptr(params_m), _ptr(params_v), _ptr(grad_params),
            _ptr(q), _ptr(q_m), _ptr(q_v), _ptr(grad_q), _ptr(score), _ptr(s_m), _ptr(s_v),
            _ptr(grad_score)), self.h)

    def fl_encode(self, params, qstep, hard_mask, header, payload, payload_words, info):
        """Fixed-length encode (header int32 [59][3]: q bits, kmin, width;
        info int64 [3]: payload bits, kept, flags)."""
        self._check(self.L.sgs_fl_encode(self.h, _ptr(params), _ptr(qstep), _ptr(hard_mask),
                                         _ptr(header), _ptr(payload), payload_words,
                                         _ptr(info)), self.h)

    def fl_decode(self, header, payload, payload_words, kept, out_pad, out):
        self._check(self.L.sgs_fl_decode(self.h, _ptr(header), _ptr(payload), payload_words,
                                         kept, out_pad, _ptr(out)), self.h)

    # ---- learned-coding stage (octree tokens, entropy coder) ----
    def octree_encode(self, params, npad, n, qstep, hard_mask, tokens, codes, dup_index,
                      dup_count, header):
        """Octree tokens of the kept positions; header: int64 [30] device
        tensor (the sgs_octree_header layout)."""
        self._check(self.L.sgs_octree_encode(
            self.h, _ptr(params), npad, n, _ptr(qstep), _ptr(hard_mask), _ptr(tokens),
            tokens.numel(), _ptr(codes), _ptr(dup_index), _ptr(dup_count),
            0 if dup_index is None else dup_index.numel(), _ptr(header)), self.h)

    @staticmethod
    def octree_header(values) -> sgs_octree_header:
        """Host header from the 30 int64 words the encoder wrote."""
        v = np.asarray(values, np.int64).reshape(-1)
        h = sgs_octree_header()
        C.memmove(C.addressof(h), v.ctypes.data, C.sizeof(h))
        return h

    def octree_decode(self, header: sgs_octree_header, tokens, dup_index, dup_count, qstep,
                      codes, xyz, out_pad, info):
        self._check(self.L.sgs_octree_decode(
            self.h, C.byref(header), _ptr(tokens), _ptr(dup_index), _ptr(dup_count),
            _ptr(qstep), _ptr(codes), _ptr(xyz), out_pad, _ptr(info)), self.h)

    def ans_max_words(self, n: int, lane_len: int) -> int:
        return int(self.L.sgs_ans_max_words(n, lane_len))

    def ans_model(self, sym, n, order, lane_len, freq, ideal_bits=None):
        self._check(self.L.sgs_ans_model(self.h, _ptr(sym), n, order, lane_len, _ptr(freq),
                                         _ptr(ideal_bits)), self.h)

    def ans_encode(self, sym, n, order, lane_len, freq, words, block_off, info):
        self._check(self.L.sgs_ans_encode(self.h, _ptr(sym), n, order, lane_len, _ptr(freq),
                                          _ptr(words), words.numel(), _ptr(block_off),
                                          _ptr(info)), self.h)

    def ans_decode(self, words, n_words, block_off, n, order, lane_len, freq, sym, info):
        self._check(self.L.sgs_ans_decode(self.h, _ptr(words), n_words, _ptr(block_off), n,
                                          order, lane_len, _ptr(freq), _ptr(sym), _ptr(info)),
                    self.h)

    def ans_decode_multi(self, streams, info):
        """streams: dicts with words, n_words, block_off, n, freq, sym, order,
        lane_len (tensors for the buffers)."""
        arr = (sgs_ans_stream * max(len(streams), 1))()
        for i, d in enumerate(streams):
            arr[i] = sgs_ans_stream(_ptr(d["words"]), d["n_words"], _ptr(d["block_off"]), d["n"],
                                    _ptr(d["freq"]), _ptr(d["sym"]), d["order"], d["lane_len"])
        self._check(self.L.sgs_ans_decode_multi(self.h, len(streams), arr, _ptr(info)), self.h)

    def morton_order(self, params, npad, n, qstep, hard_mask, header: sgs_octree_header, codes,
                     perm):
        self._check(self.L.sgs_morton_order(self.h, _ptr(params), npad, n, _ptr(qstep),
                                            _ptr(hard_mask), C.byref(header), _ptr(codes),
                                            _ptr(perm)), self.h)

    @staticmethod
    def fl_header_host(hdr) -> "C.Array":
        """Host sgs_fl_channel[59] from the encoder's int32 [59][3] header."""
        v = np.ascontiguousarray(np.asarray(hdr).reshape(59, 3), dtype=np.int32)
        arr = (sgs_fl_channel * 59)()
        C.memmove(arr, v.ctypes.data, v.nbytes)
        return arr

    @staticmethod
    def _pred(predictor):
        if predictor is None:
            return None
        v = np.ascontiguousarray(np.asarray(predictor).reshape(59), dtype=np.uint8)
        return (C.c_uint8 * 59).from_buffer_copy(v.tobytes())

    def attr_plane_rows(self, fl, predictor=None) -> int:
        r = int(self.L.sgs_attr_plane_rows(fl, self._pred(predictor)))
        if r < 0:
            raise SgsError(-1, "attr_plane_rows: bad header")
        return r

    def attr_planes(self, params, npad, perm, kept, fl, lane_len, planes, predictor=None):
        self._check(self.L.sgs_attr_planes(self.h, _ptr(params), npad, _ptr(perm), kept, fl,
                                           self._pred(predictor), lane_len, _ptr(planes)),
                    self.h)

    def attr_reconstruct(self, planes, kept, fl, lane_len, out, out_pad, predictor=None):
        self._check(self.L.sgs_attr_reconstruct(self.h, _ptr(planes), kept, fl,
                                                self._pred(predictor), lane_len, _ptr(out),
                                                out_pad), self.h)

    def positional_embedding(self, xyz, pad, count, L, d, W, b, out):
        self._check(self.L.sgs_positional_embedding(self.h, _ptr(xyz), pad, count, L, d, _ptr(W),
                                                    _ptr(b), _ptr(out)), self.h)

    def rate_variant(self, params, qstep, stats, rate_weight, out3, rate_grad=None,
                     proxy="range", masking="mult", alpha=0.0):
        o = sgs_rate_options()
        o.proxy = {"range": 0, "laplace": 1}[proxy]
        o.masking = {"mult": 0, "add": 1}[masking]
        o.alpha, o.reserved = alpha, 0
        self._check(self.L.sgs_rate_variant(self.h, _ptr(params), _ptr(qstep), _ptr(stats),
                                            C.byref(o), rate_weight, _ptr(out3),
                                            _ptr(rate_grad)), self.h)

    def rate_variant_bwd(self, params, grad_params):
        self._check(self.L.sgs_rate_variant_bwd(self.h, _ptr(params), _ptr(grad_params)), self.h)

    def ssim_loss(self, image, target, weight, loss, dL_dimage=None):
        self._check(self.L.sgs_ssim_loss(self.h, _ptr(image), _ptr(target), weight, _ptr(loss),
                                         _ptr(dL_dimage)), self.h)

    def compact(self, hard_mask, pairs, dst_pad: int) -> int:
        """Keep the Gaussians with hard_mask != 0 in every (src, dst) pair of
        device tensors ([rows][npad] -> [rows][dst_pad]); returns the kept count."""
        k = len(pairs)
        src = (C.c_void_p * k)(*[_ptr(s) for s, _ in pairs])
        dst = (C.c_void_p * k)(*[_ptr(d) for _, d in pairs])
        rows = (C.c_int32 * k)(*[1 if s.dim() == 1 else int(s.shape[0]) for s, _ in pairs])
        kept = I64()
        self._check(self.L.sgs_compact(self.h, _ptr(hard_mask), k, src, dst, rows, dst_pad,
                                       C.byref(kept)), self.h)
        return int(kept.value)

    def rate_mlp_features(self, params, qstep, stats, idx, rows, X):
        self._check(self.L.sgs_rate_mlp_features(self.h, _ptr(params), _ptr(qstep), _ptr(stats),
                                                 _ptr(idx), rows, _ptr(X)), self.h)

    def rate_mlp_infer(self, packed, theta, X, rows, out):
        self._check(self.L.sgs_rate_mlp_infer(self.h, _ptr(packed), _ptr(theta), _ptr(X), rows,
                                              _ptr(out)), self.h)

    def rate_mlp_train_scratch_bytes(self, rows) -> int:
        return int(self.L.sgs_rate_mlp_train_scratch_bytes(rows))

    def rate_mlp_train_step(self, theta, adam_m, adam_v, packed, X, target, rows, lr, step,
                            loss, grad_theta, scratch):
        self._check(self.L.sgs_rate_mlp_train_step(
            self.h, _ptr(theta), _ptr(adam_m), _ptr(adam_v), _ptr(packed), _ptr(X),
            _ptr(target), rows, lr, step, _ptr(loss), _ptr(grad_theta), _ptr(scratch)), self.h)

    def rate_mlp_train_step_static(self, theta, adam_m, adam_v, packed, X, target, rows, lr,
                                   step, loss, grad_theta):
        self._check(self.L.sgs_rate_mlp_train_step_static(
            self.h, _ptr(theta), _ptr(adam_m), _ptr(adam_v), _ptr(packed), _ptr(X),
            _ptr(target), rows, lr, step, _ptr(loss), _ptr(grad_theta)), self.h)

    def profile_enable(self, on: bool = True):
        self._check(self.L.sgs_profile_enable(self.h, 1 if on else 0), self.h)

    def profile_read(self) -> dict:
        ms = (C.c_double * len(PROF_GROUPS))()
        cnt = (C.c_int64 * len(PROF_GROUPS))()
        self._check(self.L.sgs_profile_read(self.h, ms, cnt), self.h)
        return {g: (float(ms[k]), int(cnt[k])) for k, g in enumerate(PROF_GROUPS)}
