#!/usr/bin/env python3
"""Generate the gfx950 inner step of the register-window dedispersion kernel.

The paper instantiates its kernel source from tuning parameters at run time
(Section 2.2).  Here the instantiation happens ahead of time: this script
writes ``win_asm.inc``, one inline-assembly step per (TP, DPW, NWIN,
weighted) variant, which ``engine.hip`` includes.

One step processes one input row (a channel in the forward map) for the
DPW output rows (DM trials) of one wave:

  1. load the lane's window of consecutive input samples from LDS into fixed
     VGPRs with 16-byte reads (only as many reads as the row's delay span
     needs, ``nl``);
  2. once they have landed, issue the scalar load of the next row's table
     entry (and weight), whose latency then hides behind the adds.  The loads
     go through buffer resources with a byte offset the step advances itself,
     so reads past the last row return zero instead of needing a clamp;
  3. turn VGPR index mode on and, for each of the DPW rows j, set the index
     to the row's window offset o_j (one SGPR each) and add the TP window
     registers starting at o_j into the row's TP accumulators:
        acc[j][i] += win[o_j + i]        (or fma(win[o_j + i], w, acc[j][i]))
     so each accumulator receives exactly one term per input row, in input
     row order, with one rounding per term.

The scalar unit is shared by the four SIMDs of a compute unit, so every
scalar instruction in the step costs add throughput; the step keeps them to
the index changes, the load-count tests and two waits.

A lane owns TP consecutive samples, so neighbouring lanes' windows start
4*TP bytes apart; TP/4 odd keeps the 16-byte LDS reads free of bank
conflicts.  Accumulators live in VGPRs v[ACC0 ...] and the window right
after them; the C++ side binds the accumulators with physical-register
constraints.  Table entry layout (ints): {window start, nl, o_0, ..., o_{DPW-1}}.
"""
import os
import sys

ACC0 = 32

# (TP samples per lane, DPW rows per wave, NWIN window registers)
VARIANTS = [
    (8, 8, 64),
    (16, 8, 72),
    (16, 4, 64),
    (8, 4, 48),
    (12, 4, 36),
    (12, 4, 48),
    (12, 8, 56),
    (20, 4, 44),
    (20, 8, 56),
    (28, 4, 48),
]


def entry_ints(dpw):
    n = dpw + 2
    return 4 if n <= 4 else 8 if n <= 8 else 16


def step(tp, dpw, nwin, weighted):
    """Return the C++ specialisation of win_step for one variant."""
    nacc = tp * dpw
    assert nacc % 16 == 0 and nwin % 4 == 0 and tp % 4 == 0
    w0 = ACC0 + nacc
    assert w0 + nwin <= 256
    nmin = tp // 4 + 1
    nmax = nwin // 4
    ent = entry_ints(dpw)
    lines = []
    # index mode keeps its index in M0, a register the compiler reserves for
    # itself (LDS DMA uses it): save it here and restore it at the end
    lines.append("s_mov_b32 %[m0s], m0")
    # window loads: the first nmin always, the rest while k < nl
    for k in range(nmin):
        lines.append(f"ds_read_b128 v[{w0 + 4 * k}:{w0 + 4 * k + 3}], %[addr] offset:{16 * k}")
    for k in range(nmin, nmax):
        lines.append(f"s_cmp_le_u32 %[nl], {k}")
        lines.append("s_cbranch_scc1 .Lwin_loaded_%=")
        lines.append(f"ds_read_b128 v[{w0 + 4 * k}:{w0 + 4 * k + 3}], %[addr] offset:{16 * k}")
    lines.append(".Lwin_loaded_%=:")
    lines.append("s_waitcnt lgkmcnt(0)")
    # the next row's table entry (and weight) load while the adds run; the
    # final wait leaves them complete when the step returns
    lines.append(f"s_buffer_load_dwordx{ent} %[nxt], %[trs], %[toff]")
    lines.append(f"s_add_u32 %[toff], %[toff], {4 * ent}")
    if weighted:
        lines.append("s_buffer_load_dword %[wn], %[wrs], %[woff]")
        lines.append("s_add_u32 %[woff], %[woff], 4")
    for j in range(dpw):
        if j == 0:
            lines.append("s_set_gpr_idx_on %[o0], gpr_idx(SRC0)")
        else:
            lines.append(f"s_set_gpr_idx_idx %[o{j}]")
        for i in range(tp):
            a = ACC0 + j * tp + i
            if weighted:
                lines.append(f"v_fma_f32 v{a}, v{w0 + i}, %[w], v{a}")
            else:
                lines.append(f"v_add_f32 v{a}, v{w0 + i}, v{a}")
    lines.append("s_set_gpr_idx_off")
    lines.append("s_mov_b32 m0, %[m0s]")
    lines.append("s_waitcnt lgkmcnt(0)")
    asm = "".join(f'    "{ln}\\n\\t"\n' for ln in lines)
    outs = ['[m0s] "=&s"(m0s)', '[nxt] "=&s"(nxt)', '[toff] "+s"(toff)']
    if weighted:
        outs.append('[wn] "=&s"(wn)')
        outs.append('[woff] "+s"(woff)')
    for q in range(nacc // 16):
        lo = ACC0 + 16 * q
        outs.append(f'[a{q}] "+{{v[{lo}:{lo + 15}]}}"(acc[{q}])')
    ins = ['[addr] "v"(addr)', '[nl] "s"(cur[1])', '[trs] "s"(trs)']
    for j in range(dpw):
        ins.append(f'[o{j}] "s"(cur[{2 + j}])')
    if weighted:
        ins.append('[w] "s"(w)')
        ins.append('[wrs] "s"(wrs)')
    clob = [f'"v{w0 + r}"' for r in range(nwin)] + ['"scc"']
    wflag = "true" if weighted else "false"
    etype = f"ent{ent}_t"
    return (
        f"template <>\n"
        f"__device__ __forceinline__ void win_step<{tp}, {dpw}, {nwin}, {wflag}>(v16f* acc, uint32_t addr,\n"
        f"    const {etype}& cur, {etype}& nxt, __amdgpu_buffer_rsrc_t trs, uint32_t& toff, float w,\n"
        f"    float& wn, __amdgpu_buffer_rsrc_t wrs, uint32_t& woff) {{\n"
        f"  uint32_t m0s;\n"
        f"  (void)w;\n"
        f"  (void)wn;\n"
        f"  (void)wrs;\n"
        f"  (void)woff;\n"
        f"  asm volatile(\n{asm}"
        f"    : {', '.join(outs)}\n"
        f"    : {', '.join(ins)}\n"
        f"    : {', '.join(clob)});\n"
        f"}}\n"
    )


SGPR_A = 40  # entry sets of the pass block live in fixed SGPRs from here


def pass_block(tp, dpw, nwin, cc, weighted):
    """Specialisation of WinPass: the rows of one LDS pass in one block with
    VGPR index mode on throughout (turning it on and off costs about as much
    as 30 adds; changing the index is nearly free).  Vector instructions other
    than the adds take their first operand from an SGPR or a literal, so the
    index does not touch them.  Row r sums from entry set A (r even) or B (r
    odd), both in fixed SGPRs, and loads the next row's entry into the other
    set; on exit the next pass's first entry is in A."""
    nacc = tp * dpw
    w0 = ACC0 + nacc
    assert w0 + nwin <= 256
    nmin = tp // 4 + 1
    nmax = nwin // 4
    ent = entry_ints(dpw)
    sa, sb = SGPR_A, SGPR_A + ent
    L = ["s_mov_b32 %[m0s], m0", f"s_set_gpr_idx_on s{sa + 2}, gpr_idx(SRC0)"]
    for r in range(cc):
        X, Y = (sa, sb) if r % 2 == 0 else (sb, sa)
        wX, wY = ("%[wa]", "%[wb]") if r % 2 == 0 else ("%[wb]", "%[wa]")
        L.append(f"s_lshl_b32 %[t], s{X}, 2")
        L.append("v_add_u32 %[va], %[t], %[vrow]")
        for k in range(nmin):
            L.append(f"ds_read_b128 v[{w0 + 4 * k}:{w0 + 4 * k + 3}], %[va] offset:{16 * k}")
        for k in range(nmin, nmax):
            L.append(f"s_cmp_le_u32 s{X + 1}, {k}")
            L.append(f"s_cbranch_scc1 .Lr{r}_loaded_%=")
            L.append(f"ds_read_b128 v[{w0 + 4 * k}:{w0 + 4 * k + 3}], %[va] offset:{16 * k}")
        L.append(f".Lr{r}_loaded_%=:")
        L.append("s_waitcnt lgkmcnt(0)")
        L.append(f"s_buffer_load_dwordx{ent} s[{Y}:{Y + ent - 1}], %[trs], %[toff]")
        L.append(f"s_add_u32 %[toff], %[toff], {4 * ent}")
        if weighted:
            L.append(f"s_buffer_load_dword {wY}, %[wrs], %[woff]")
            L.append("s_add_u32 %[woff], %[woff], 4")
        for j in range(dpw):
            if not (r == 0 and j == 0):
                L.append(f"s_set_gpr_idx_idx s{X + 2 + j}")
            for i in range(tp):
                a = ACC0 + j * tp + i
                if weighted:
                    L.append(f"v_fma_f32 v{a}, v{w0 + i}, {wX}, v{a}")
                else:
                    L.append(f"v_add_f32 v{a}, v{w0 + i}, v{a}")
        L.append("v_add_u32 %[vrow], %[rowbytes], %[vrow]")
        L.append("s_waitcnt lgkmcnt(0)")
        if r + 1 < cc:
            L.append(f"s_cmp_le_u32 %[ncc], {r + 1}")
            L.append(f"s_cbranch_scc1 {'.Lcopy_%=' if r % 2 == 0 else '.Lend_%='}")
    if cc % 2 == 0:  # after the last (odd) row the next entry is already in A
        L.append("s_branch .Lend_%=")
    L.append(".Lcopy_%=:")
    for q in range(0, ent, 2):
        L.append(f"s_mov_b64 s[{sa + q}:{sa + q + 1}], s[{sb + q}:{sb + q + 1}]")
    if weighted:
        L.append("s_mov_b32 %[wa], %[wb]")
    L.append(".Lend_%=:")
    L.append("s_set_gpr_idx_off")
    L.append("s_mov_b32 m0, %[m0s]")
    asm = "".join(f'    "{ln}\\n\\t"\n' for ln in L)
    etype = f"ent{ent}_t"
    outs = ['[m0s] "=&s"(m0s)', '[t] "=&s"(t)', '[va] "=&v"(va)', '[vrow] "+v"(vrow)', '[toff] "+s"(toff)',
            f'[ea] "+{{s[{sa}:{sa + ent - 1}]}}"(ea)', f'[eb] "=&{{s[{sb}:{sb + ent - 1}]}}"(eb)']
    if weighted:
        outs += ['[wa] "+s"(wa)', '[wb] "=&s"(wb)', '[woff] "+s"(woff)']
    for q in range(nacc // 16):
        lo = ACC0 + 16 * q
        outs.append(f'[acc{q}] "+{{v[{lo}:{lo + 15}]}}"(acc[{q}])')
    ins = ['[ncc] "s"(ncc)', '[trs] "s"(trs)', '[rowbytes] "i"(ROWCAP * 4)']
    if weighted:
        ins.append('[wrs] "s"(wrs)')
    clob = [f'"v{w0 + r}"' for r in range(nwin)] + ['"scc"']
    wflag = "true" if weighted else "false"
    return (
        f"template <int ROWCAP>\n"
        f"struct WinPass<{tp}, {dpw}, {nwin}, {cc}, {wflag}, ROWCAP> {{\n"
        f"  static __device__ __forceinline__ void run(v16f* acc, uint32_t& vrow, int ncc, {etype}& ea,\n"
        f"      __amdgpu_buffer_rsrc_t trs, uint32_t& toff, float& wa, __amdgpu_buffer_rsrc_t wrs, uint32_t& woff) {{\n"
        f"    uint32_t m0s, t, va;\n"
        f"    {etype} eb;\n"
        f"    float wb;\n"
        f"    (void)wa;\n"
        f"    (void)wb;\n"
        f"    (void)wrs;\n"
        f"    (void)woff;\n"
        f"    asm volatile(\n{asm}"
        f"      : {', '.join(outs)}\n"
        f"      : {', '.join(ins)}\n"
        f"      : {', '.join(clob)});\n"
        f"  }}\n"
        f"}};\n"
    )


def jmp_block_bytes(tp):
    """Bytes of one static block of the jump form: TP two-operand adds (or
    fmacs) of 4 bytes each and the 4-byte jump to the next block."""
    return 4 * tp + 4


def jmp_pass(tp, dpw, nwin, cc, weighted, full=False, acc0=ACC0):
    """Specialisation of JmpPass: the rows of one LDS pass without VGPR index
    mode.  Each DM slot j has a region of static blocks, one per window
    offset o (0 <= o <= NWIN - TP); block (j, o) adds window registers
    o .. o + TP - 1 into slot j's accumulators and jumps to slot j + 1's
    chosen block (the last slot returns).  Per row the table entry holds, for
    every slot, the byte offset o * BLK of its block inside the slot's region,
    so a row costs one scalar add and one jump per slot instead of indexed
    operands (which issue about 1.7 times slower on gfx950).  A slot's target
    is its own region's base plus the entry's offset: whatever the entry
    holds, slot j can only reach slot j's blocks, so the chain always moves on
    to the next slot.

    The targets' high words are the region's when the region does not cross
    a 4 GB boundary (checked once per pass); otherwise a second copy of the
    rows propagates the carries.  Entry sets alternate between two fixed
    SGPR ranges as in the index-mode pass.  The accumulators start at
    v[acc0]: a low acc0 leaves the fewest registers to the compiler and lets
    small shapes reach 4 waves per SIMD."""
    nacc = tp * dpw
    w0 = acc0 + nacc
    assert w0 + nwin <= 256
    nmin = tp // 4 + 1
    nmax = nwin // 4
    ent = entry_ints(dpw)
    noff = nwin - tp + 1
    blk = jmp_block_bytes(tp)
    slot = noff * blk
    region = dpw * slot
    # an entry's dpw + 2 used ints load as power-of-two pieces (4-aligned
    # destinations for 4 and 8 dwords)
    used = dpw + 2
    pieces = []
    k = 0
    for n in (8, 4, 2, 1):
        while used - k >= n:
            pieces.append((k, n))
            k += n
    sa = SGPR_A                # set A: bound to the C++ entry (ent ints)
    sb = sa + ent              # set B: used ints only, clobbered
    tg = sb + ((used + 1) // 2) * 2   # targets: one SGPR pair per slot
    sl = tg + 2 * dpw          # low word of each slot's region base
    ret = sl + dpw + (dpw % 2)
    base = ret + 2
    wreg = base + 2            # weight of the row being summed (weighted form)
    top = wreg + (1 if weighted else 0)
    # s100 and up are reserved on gfx950
    assert top <= 96 and tg % 2 == 0 and ret % 2 == 0 and base % 2 == 0 and sb % 4 == 0

    def load_entry(dst):
        for k0, n in pieces:
            op = "s_buffer_load_dword" if n == 1 else f"s_buffer_load_dwordx{n}"
            reg = f"s{dst + k0}" if n == 1 else f"s[{dst + k0}:{dst + k0 + n - 1}]"
            L.append(f"{op} {reg}, %[trs], %[toff] offset:{4 * k0}")
        L.append(f"s_add_u32 %[toff], %[toff], {4 * ent}")

    L = [f"s_getpc_b64 s[{base}:{base + 1}]", ".Lpc_%=:",
         f"s_add_u32 s{base}, s{base}, .Lregion_%= - .Lpc_%=",
         f"s_addc_u32 s{base + 1}, s{base + 1}, 0"]
    for j in range(dpw):
        L.append(f"s_add_u32 s{sl + j}, s{base}, {j * slot}")
    # carry out of the region's last byte: take the rows that propagate it
    L.append(f"s_add_u32 s{ret}, s{base}, {region}")
    L.append("s_cbranch_scc1 .Lslow_%=")
    for j in range(dpw):
        L.append(f"s_mov_b32 s{tg + 2 * j + 1}, s{base + 1}")

    def rows(path):
        for r in range(cc):
            X, Y = (sa, sb) if r % 2 == 0 else (sb, sa)
            wX, wY = ("%[wa]", "%[wb]") if r % 2 == 0 else ("%[wb]", "%[wa]")
            L.append(f"s_lshl_b32 %[t], s{X}, 2")
            L.append("v_add_u32 %[va], %[t], %[vrow]")
            for k in range(nmin):
                L.append(f"ds_read_b128 v[{w0 + 4 * k}:{w0 + 4 * k + 3}], %[va] offset:{16 * k}")
            for k in range(nmin, nmax):
                if not full:
                    L.append(f"s_cmp_le_u32 s{X + 1}, {k}")
                    L.append(f"s_cbranch_scc1 .L{path}{r}_loaded_%=")
                L.append(f"ds_read_b128 v[{w0 + 4 * k}:{w0 + 4 * k + 3}], %[va] offset:{16 * k}")
            L.append(f".L{path}{r}_loaded_%=:")
            L.append("s_waitcnt lgkmcnt(0)")
            load_entry(Y)
            if weighted:
                L.append(f"s_mov_b32 s{wreg}, {wX}")
                L.append(f"s_buffer_load_dword {wY}, %[wrs], %[woff]")
                L.append("s_add_u32 %[woff], %[woff], 4")
            for j in range(dpw):
                if path == "f":
                    L.append(f"s_add_u32 s{tg + 2 * j}, s{sl + j}, s{X + 2 + j}")
                else:
                    L.append(f"s_add_u32 s{tg + 2 * j}, s{base}, s{X + 2 + j}")
                    L.append(f"s_addc_u32 s{tg + 2 * j + 1}, s{base + 1}, 0")
                    L.append(f"s_add_u32 s{tg + 2 * j}, s{tg + 2 * j}, {j * slot}")
                    L.append(f"s_addc_u32 s{tg + 2 * j + 1}, s{tg + 2 * j + 1}, 0")
            L.append(f"s_swappc_b64 s[{ret}:{ret + 1}], s[{tg}:{tg + 1}]")
            L.append("v_add_u32 %[vrow], %[rowbytes], %[vrow]")
            L.append("s_waitcnt lgkmcnt(0)")
            if r + 1 < cc:
                L.append(f"s_cmp_le_u32 %[ncc], {r + 1}")
                L.append(f"s_cbranch_scc1 {'.Lcopy_%=' if r % 2 == 0 else '.Lend_%='}")
        if cc % 2 == 0:  # after the last (odd) row the next entry is already in A
            L.append("s_branch .Lend_%=")
        else:
            L.append("s_branch .Lcopy_%=")

    rows("f")
    L.append(".Lslow_%=:")
    rows("s")
    L.append(".Lcopy_%=:")
    for q in range(0, used, 2):
        L.append(f"s_mov_b64 s[{sa + q}:{sa + q + 1}], s[{sb + q}:{sb + q + 1}]")
    if weighted:
        L.append("s_mov_b32 %[wa], %[wb]")
    L.append("s_branch .Lend_%=")
    L.append(".Lregion_%=:")
    for j in range(dpw):
        nxt = f"s[{tg + 2 * (j + 1)}:{tg + 2 * (j + 1) + 1}]" if j + 1 < dpw else f"s[{ret}:{ret + 1}]"
        for o in range(noff):
            for i in range(tp):
                a = acc0 + j * tp + i
                if weighted:
                    L.append(f"v_fmac_f32 v{a}, s{wreg}, v{w0 + o + i}")
                else:
                    L.append(f"v_add_f32 v{a}, v{w0 + o + i}, v{a}")
            L.append(f"s_setpc_b64 {nxt}")
    L.append(".Lregion_end_%=:")
    # the host computes block offsets as o * BLK: the assembled region must match
    L.append(f".if .Lregion_end_%= - .Lregion_%= - {region}")
    L.append(".error \\\"jump region size differs from the block layout\\\"")
    L.append(".endif")
    L.append(".Lend_%=:")
    asm = "".join(f'    "{ln}\\n\\t"\n' for ln in L)
    etype = f"ent{ent}_t"
    outs = ['[t] "=&s"(t)', '[va] "=&v"(va)', '[vrow] "+v"(vrow)', '[toff] "+s"(toff)',
            f'[ea] "+{{s[{sa}:{sa + ent - 1}]}}"(ea)']
    if weighted:
        outs += ['[wa] "+s"(wa)', '[wb] "=&s"(wb)', '[woff] "+s"(woff)']
    for q in range(nacc // 16):
        lo = acc0 + 16 * q
        outs.append(f'[acc{q}] "+{{v[{lo}:{lo + 15}]}}"(acc[{q}])')
    ins = ['[ncc] "s"(ncc)', '[trs] "s"(trs)', '[rowbytes] "i"(ROWCAP * 4)']
    if weighted:
        ins.append('[wrs] "s"(wrs)')
    clob = [f'"v{w0 + r}"' for r in range(nwin)] + [f'"s{r}"' for r in range(sb, top)] + ['"scc"']
    wflag = "true" if weighted else "false"
    return (
        f"template <int ROWCAP>\n"
        f"struct JmpPass<{tp}, {dpw}, {nwin}, {cc}, {wflag}, {'true' if full else 'false'}, ROWCAP> {{\n"
        f"  static __device__ __forceinline__ void run(v16f* acc, uint32_t& vrow, int ncc, {etype}& ea,\n"
        f"      __amdgpu_buffer_rsrc_t trs, uint32_t& toff, float& wa, __amdgpu_buffer_rsrc_t wrs, uint32_t& woff) {{\n"
        f"    uint32_t t, va;\n"
        f"    float wb;\n"
        f"    (void)wa;\n"
        f"    (void)wb;\n"
        f"    (void)wrs;\n"
        f"    (void)woff;\n"
        f"    asm volatile(\n{asm}"
        f"      : {', '.join(outs)}\n"
        f"      : {', '.join(ins)}\n"
        f"      : {', '.join(clob)});\n"
        f"  }}\n"
        f"}};\n"
    )


# (TP, DPW, NWIN, CC[, first accumulator VGPR]) combinations with a jump-form pass
JMP_VARIANTS = [
    (20, 4, 44, 4),
    (20, 8, 56, 4),
    (20, 8, 56, 6),
    (28, 4, 48, 4),
    (12, 4, 36, 4),
    (20, 4, 40, 3, 8),
    (20, 4, 40, 6, 8),
    (20, 4, 40, 8, 8),
    (20, 4, 40, 10, 8),
    (20, 4, 44, 8, 4),
    (20, 4, 44, 10, 4),
]


# (TP, DPW, NWIN, CC) combinations that get a whole-pass block
PASS_VARIANTS = [
    (12, 4, 36, 4),
    (12, 8, 56, 4),
    (20, 4, 44, 4),
    (20, 8, 56, 4),
    (20, 8, 56, 6),
    (28, 4, 48, 4),
]


def main(out_path):
    parts = [
        "// Generated by gen_win_asm.py: inner step of the register-window kernel.\n",
        "// Do not edit by hand.\n",
        "#pragma once\n\n",
        f"#define WIN_ACC0 {ACC0}\n\n",
        "// Table entry of one (wave tile, input row): {window start, loads, offset per row...}.\n",
        "typedef int32_t ent4_t __attribute__((ext_vector_type(4)));\n",
        "typedef int32_t ent8_t __attribute__((ext_vector_type(8)));\n",
        "typedef int32_t ent16_t __attribute__((ext_vector_type(16)));\n",
        "template <int DPW> struct EntT {\n",
        "  typedef typename std::conditional<(DPW + 2 <= 4), ent4_t,\n",
        "      typename std::conditional<(DPW + 2 <= 8), ent8_t, ent16_t>::type>::type type;\n",
        "  static constexpr int ints = DPW + 2 <= 4 ? 4 : DPW + 2 <= 8 ? 8 : 16;\n",
        "};\n\n",
        "// Sums the current row (entry cur, weight w) from its window at LDS byte\n",
        "// address addr, and loads the next row's entry into nxt from the table\n",
        "// resource trs at byte offset toff (and its weight into wn from wrs at\n",
        "// woff), advancing both offsets by one row.\n",
        "template <int TP, int DPW, int NWIN, bool WEIGHTED>\n",
        "__device__ __forceinline__ void win_step(v16f* acc, uint32_t addr, const typename EntT<DPW>::type& cur,\n",
        "    typename EntT<DPW>::type& nxt, __amdgpu_buffer_rsrc_t trs, uint32_t& toff, float w, float& wn,\n",
        "    __amdgpu_buffer_rsrc_t wrs, uint32_t& woff);\n\n",
    ]
    for tp, dpw, nwin in VARIANTS:
        for weighted in (False,):
            parts.append(step(tp, dpw, nwin, weighted))
            parts.append("\n")
    parts += [
        "// Runs the rows of one LDS pass (ncc <= CC rows) with index mode on\n",
        "// throughout: vrow is this lane's byte address in the pass's first row slot\n",
        "// (advanced by one row per row), ea the first row's entry on entry and the\n",
        "// next pass's on exit, wa likewise for the weight.\n",
        "template <int TP, int DPW, int NWIN, int CC, bool WEIGHTED, int ROWCAP>\n",
        "struct WinPass;\n",
        "template <int TP, int DPW, int NWIN, int CC>\n",
        "struct HasWinPass : std::false_type {};\n",
    ]
    for tp, dpw, nwin, cc in PASS_VARIANTS:
        parts.append(f"template <> struct HasWinPass<{tp}, {dpw}, {nwin}, {cc}> : std::true_type {{}};\n")
    parts.append("\n")
    for tp, dpw, nwin, cc in PASS_VARIANTS:
        for weighted in (False,):
            parts.append(pass_block(tp, dpw, nwin, cc, weighted))
            parts.append("\n")
    parts += [
        "// Jump form of a pass (no index mode): same interface as WinPass; the\n",
        "// table entry's per-row values are block offsets o * JmpBlockBytes<TP>.\n",
        "template <int TP, int DPW, int NWIN, int CC, bool WEIGHTED, bool FULL, int ROWCAP>\n",
        "struct JmpPass;\n",
        "template <int TP, int DPW, int NWIN, int CC>\n",
        "struct HasJmpPass : std::false_type {};\n",
        "template <int TP> constexpr int JmpBlockBytes = 4 * TP + 4;\n",
        "// first accumulator VGPR of a jump-form pass\n",
        "template <int TP, int DPW, int NWIN, int CC>\n",
        "struct JmpAcc0 { static constexpr int value = 0; };\n",
    ]
    for jv in JMP_VARIANTS:
        tp, dpw, nwin, cc = jv[:4]
        acc0 = jv[4] if len(jv) > 4 else ACC0
        assert jmp_block_bytes(tp) == 4 * tp + 4
        parts.append(f"template <> struct HasJmpPass<{tp}, {dpw}, {nwin}, {cc}> : std::true_type {{}};\n")
        parts.append(f"template <> struct JmpAcc0<{tp}, {dpw}, {nwin}, {cc}> {{ static constexpr int value = {acc0}; }};\n")
    parts.append("\n")
    for jv in JMP_VARIANTS:
        tp, dpw, nwin, cc = jv[:4]
        acc0 = jv[4] if len(jv) > 4 else ACC0
        for weighted in (False,):
            for full in (False, True):
                parts.append(jmp_pass(tp, dpw, nwin, cc, weighted, full, acc0))
                parts.append("\n")
    text = "".join(parts)
    if os.path.exists(out_path) and open(out_path).read() == text:
        return
    with open(out_path, "w") as f:
        f.write(text)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else os.path.join(os.path.dirname(os.path.abspath(__file__)), "win_asm.inc"))
