"""Device-side helpers: upload a batch to HBM with torch, run the libss kernels.

Marshalling only.  Torch supplies device memory and the stream; every
encoding and filtering step is a libss.so kernel.
"""
from __future__ import annotations

import numpy as np
import torch

from . import (ss_create, ss_filter_ascii_async, ss_filter_submaze_async, ss_select_accepted_async, ss_verify_async,
               ss_verify_banded_async, ss_filter_plain_async, ss_filter_sliced_async, ss_filter_sliced_range_async,
               ss_filter_wave_async, ss_pack_sliced_async, ss_pack_stream_async, ss_sliced_bytes, ss_stream_words)

_ctx = {}


def context(device: int = 0) -> int:
    if device not in _ctx:
        _ctx[device] = ss_create(device)
    return _ctx[device]


def _dev(device):
    return torch.device("cuda", device)


class DeviceBatch:
    """A batch of pairs resident in HBM (ASCII reads/refs, offsets, lengths, per-pair E)."""

    def __init__(self, batch: dict, device: int = 0):
        d = _dev(device)
        self.device = device
        self.n = int(batch["n"]) if "n" in batch else len(batch["lengths"])
        self.lengths_np = np.ascontiguousarray(batch["lengths"], dtype=np.int32)
        self.offsets_np = np.ascontiguousarray(batch["offsets"], dtype=np.int64)
        self.total = int(len(batch["reads"]))
        # pad ASCII buffers to 16 bytes so vector loads of the encoder stay inside
        pad = (-self.total) % 16 + 16
        self.reads = torch.empty(self.total + pad, dtype=torch.uint8, device=d)
        self.refs = torch.empty(self.total + pad, dtype=torch.uint8, device=d)
        self.reads[self.total:].fill_(ord("A"))
        self.refs[self.total:].fill_(ord("A"))
        if self.total:
            self.reads[: self.total].copy_(torch.from_numpy(np.ascontiguousarray(batch["reads"])))
            self.refs[: self.total].copy_(torch.from_numpy(np.ascontiguousarray(batch["refs"])))
        self.offsets = torch.from_numpy(self.offsets_np).to(d)
        self.lengths = torch.from_numpy(self.lengths_np).to(d)
        E = batch.get("E")
        self.E_np = None if E is None else np.ascontiguousarray(E, dtype=np.int32)
        self.E = None if E is None else torch.from_numpy(self.E_np).to(d)
        self.uniform_m = int(self.lengths_np[0]) if self.n and np.all(self.lengths_np == self.lengths_np[0]) else None
        # pairs stored back to back (pair i at byte i*m): the encoder can stream them
        self.contiguous = self.uniform_m is not None and bool(
            np.array_equal(self.offsets_np, np.arange(self.n, dtype=np.int64) * self.uniform_m))
        self.err = torch.zeros(1, dtype=torch.int32, device=d)

    # ---- encodings -------------------------------------------------------------
    def pack_sliced(self, index=None, m=None, n=None, stream=None, packed=None) -> torch.Tensor:
        """Lane-sliced encoding of all pairs (or of the pairs listed in index, all of length m)."""
        n = self.n if n is None else n
        m = self.uniform_m if m is None else m
        if m is None:
            raise ValueError("lane-sliced encoding needs pairs of one length")
        words = max(4, ss_sliced_bytes(n, m) // 4)
        if packed is None:
            packed = torch.empty(words, dtype=torch.int32, device=_dev(self.device))
        assert packed.numel() >= words
        offsets = None if (index is None and self.contiguous) else self.offsets
        ss_pack_sliced_async(context(self.device), self.reads, self.refs, offsets, index, n, m, packed,
                             self.err, stream or torch.cuda.current_stream(self.device))
        return packed

    def pack_stream(self, stream=None, packed=None) -> torch.Tensor:
        words = 4 * ss_stream_words(self.total)
        if packed is None:
            packed = torch.empty(words, dtype=torch.int32, device=_dev(self.device))
        assert packed.numel() >= words
        ss_pack_stream_async(context(self.device), self.reads, self.refs, self.total, packed, self.err,
                             stream or torch.cuda.current_stream(self.device))
        return packed

    def err_bits(self) -> int:
        """The error word the encoders and the fused kernel OR into: bit 0 a byte outside ACGTacgt,
        bit 1 a bounded wait between the fused kernel's wavefronts that gave up."""
        return int(self.err.item())

    def bad_bases(self) -> bool:
        return bool(self.err_bits() & 1)

    def wait_gave_up(self) -> bool:
        return bool(self.err_bits() & 2)

    def check_err(self, where: str) -> None:
        """Raise if the error word is set (either bit): results written since it was cleared are
        unspecified."""
        e = self.err_bits()
        if e:
            what = []
            if e & 1:
                what.append("byte outside ACGTacgt")
            if e & 2:
                what.append("a wait inside the fused kernel gave up")
            raise RuntimeError(f"{where}: error word {e:#x} ({', '.join(what) or 'unknown bit'})")

    # ---- filters ---------------------------------------------------------------
    def new_out(self, n=None) -> torch.Tensor:
        return torch.empty(max(8, self.n if n is None else n), dtype=torch.int16, device=_dev(self.device))

    def filter_sliced(self, packed, E: int, out=None, n=None, m=None, stream=None) -> torch.Tensor:
        n = self.n if n is None else n
        m = self.uniform_m if m is None else m
        out = self.new_out(n) if out is None else out
        ss_filter_sliced_async(context(self.device), packed, n, m, E, out,
                               stream or torch.cuda.current_stream(self.device))
        return out

    def filter_sliced_range(self, packed, E_lo: int, E_hi: int, out=None, stream=None) -> torch.Tensor:
        """Results of every threshold E_lo..E_hi: row E - E_lo of the returned (E_hi - E_lo + 1, stride)
        tensor holds threshold E's n result words."""
        stride = (self.n + 7) // 8 * 8
        if out is None:
            out = torch.empty((E_hi - E_lo + 1, stride), dtype=torch.int16, device=_dev(self.device))
        ss_filter_sliced_range_async(context(self.device), packed, self.n, self.uniform_m, E_lo, E_hi, out, stride,
                                     stream or torch.cuda.current_stream(self.device))
        return out

    def filter_submaze(self, packed, E: int, sub_width: int, out=None, stream=None) -> torch.Tensor:
        """Snake-on-Chip sub-mazes of sub_width columns over the lane-sliced encoding."""
        out = self.new_out() if out is None else out
        ss_filter_submaze_async(context(self.device), packed, self.n, self.uniform_m, E, sub_width, out,
                                stream or torch.cuda.current_stream(self.device))
        return out

    def filter_fused(self, E: int, out=None, tile_groups: int = 0, stream=None) -> torch.Tensor:
        """Encode and filter in one call (pairs of one length stored back to back): fused kernel or chunks."""
        if not self.contiguous:
            raise ValueError("the fused kernel needs pairs of one length stored back to back")
        out = self.new_out() if out is None else out
        ss_filter_ascii_async(context(self.device), self.reads, self.refs, self.n, self.uniform_m, E, tile_groups,
                              out, self.err, stream or torch.cuda.current_stream(self.device))
        return out

    def filter_plain(self, packed, E: int, per_pair: bool = False, out=None, stream=None) -> torch.Tensor:
        out = self.new_out() if out is None else out
        ss_filter_plain_async(context(self.device), packed, self.total, self.offsets, self.lengths,
                              self.E if per_pair else None, self.n, E, out,
                              stream or torch.cuda.current_stream(self.device))
        return out

    def filter_wave(self, packed, E: int, per_pair: bool = False, out=None, stream=None) -> torch.Tensor:
        out = self.new_out() if out is None else out
        ss_filter_wave_async(context(self.device), packed, self.total, self.offsets, self.lengths,
                             self.E if per_pair else None, self.n, E, out,
                             stream or torch.cuda.current_stream(self.device))
        return out


    # ---- verification -----------------------------------------------------------
    def verify(self, packed, index=None, n=None, max_len=None, out=None, stream=None) -> torch.Tensor:
        """Exact edit distance of the listed pairs (all pairs when index is None), int32 per entry."""
        n = (self.n if index is None else int(index.numel())) if n is None else n
        max_len = int(self.lengths_np.max()) if max_len is None and self.n else (max_len or 0)
        out = torch.empty(max(1, n), dtype=torch.int32, device=_dev(self.device)) if out is None else out
        ss_verify_async(context(self.device), packed, self.total, self.offsets, self.lengths, index, n, max_len, out,
                        stream or torch.cuda.current_stream(self.device))
        return out

    def verify_banded(self, packed, E: int, per_pair: bool = False, index=None, n=None, out=None,
                      stream=None) -> torch.Tensor:
        """Edit distance when within the threshold (per pair, or E), else threshold + 1; int32 per entry."""
        n = (self.n if index is None else int(index.numel())) if n is None else n
        out = torch.empty(max(1, n), dtype=torch.int32, device=_dev(self.device)) if out is None else out
        ss_verify_banded_async(context(self.device), packed, self.total, self.offsets, self.lengths,
                               self.E if per_pair else None, E, index, n, out,
                               stream or torch.cuda.current_stream(self.device))
        return out

    def select_accepted(self, results, index_out=None, count=None, stream=None):
        """(index tensor, count tensor) of the pairs whose result word has the accept bit."""
        d = _dev(self.device)
        index_out = torch.empty(max(1, self.n), dtype=torch.int64, device=d) if index_out is None else index_out
        count = torch.empty(1, dtype=torch.int64, device=d) if count is None else count
        ss_select_accepted_async(context(self.device), results, self.n, index_out, count,
                                 stream or torch.cuda.current_stream(self.device))
        return index_out, count


def results_numpy(out: torch.Tensor, n: int):
    """(accept uint8[n], edits int32[n]) from a device result tensor."""
    r = out[:n].cpu().numpy().view(np.uint16)
    return (r >> 15).astype(np.uint8), (r & 0x7FFF).astype(np.int32)
