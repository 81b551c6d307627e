"""MI355X (gfx950) AES for very many independent 16-byte blocks.

Kepner et al., "Parallel Vectorized Algebraic AES in MATLAB ..." (arXiv
1506.08503) frames AES as GF(2^8) algebra vectorized over many messages; this
package runs that cipher (ECB and CTR, the paper's CBC over a message matrix,
and GCM; 128/192/256-bit keys) as hand-written HIP kernels behind the C ABI in
``include/aesmi.h``.  ``aesmi`` is the thin
Python binding; ``batch`` and ``serve`` add many-message batching and a
continuous-batching request loop on top (``serve.run_native`` runs the loop
in the library, ``serve.Server`` is the same loop in Python).
"""
from .aesmi import (AesError, KeySchedule, Launch, Segment, BatchTune, lib, expand_key,
                    schedule_to_device, key_schedule, expand_keys_device, ecb_encrypt,
                    ecb_decrypt, ctr_xcrypt, cbc_encrypt, cbc_decrypt, gcm_encrypt, gcm_decrypt, ghash,
                    gcm_workspace_bytes, ghash_workspace_bytes, device_cu_count, header_functions,
                    LAYOUT_AUTO, LAYOUT_TTABLE, LAYOUT_BITSLICE, SCHEDULE_BYTES,
                    SEGMENT_BYTES, STATUS, segment_dtype, batched_workspace_bytes,
                    ctr_xcrypt_batched, ctr_xcrypt_batched_noalloc, NOALLOC_MAX_SEGS,
                    batched_read_status, BatchedGraph, ServeParams, ServeStats,
                    serve_request_dtype)

__all__ = ["AesError", "KeySchedule", "Launch", "Segment", "BatchTune", "lib", "expand_key",
           "schedule_to_device", "key_schedule", "expand_keys_device", "ecb_encrypt",
           "ecb_decrypt", "ctr_xcrypt", "cbc_encrypt", "cbc_decrypt", "gcm_encrypt", "gcm_decrypt",
           "ghash", "gcm_workspace_bytes", "ghash_workspace_bytes", "device_cu_count", "header_functions",
           "LAYOUT_AUTO", "LAYOUT_TTABLE", "LAYOUT_BITSLICE", "SCHEDULE_BYTES",
           "SEGMENT_BYTES", "STATUS", "segment_dtype", "batched_workspace_bytes",
           "ctr_xcrypt_batched", "ctr_xcrypt_batched_noalloc", "NOALLOC_MAX_SEGS",
           "batched_read_status", "BatchedGraph", "ServeParams", "ServeStats",
           "serve_request_dtype"]
