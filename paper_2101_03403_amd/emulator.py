"""Instruction-set emulator front-end over encrypted data (Sec. 4, 6).

A load/store machine in the style of the paper's CryptoEmu: the program is
cleartext assembly, the data is encrypted.

* **Registers.** vRegs hold W encrypted bits each, and NZCV is one more
  4-bit vReg. Together with the HE data memory they live in device
  ciphertext pools.
* **Fetch and decode.** The cleartext PC fetches an instruction and decodes
  it. Each data-processing instruction runs its gate circuit (from
  ``circuits``) through the level scheduler on the GPU.
* **Flag-setting forms.** ADDS, SUBS and CMP also evaluate the NZCV circuit
  (Sec. 6.1).
* **Branches.** A conditional branch asks the client, who holds the secret
  key, to decide from the encrypted flags (Sec. 4.2, 6.2). The client here is
  a callback, and ``make_client`` builds one from a secret key.

Instruction set (operands: Rd, Rn, and Rm or #imm), following the paper's
listings:

    MOV Rd, Rn, #imm | MOV Rd, Rm        MVN Rd, Rm
    LOAD Rd, addr    | STORE Rs, addr    (addr: word index into HE data memory)
    ADD/ADDS/SUB/SUBS/MUL/UDIV/AND/ORR/EOR/ORN Rd, Rn, Rm|#imm
    LSL|LLS, LSR|LRS, ASR|ARS Rd, Rn, Rm|#imm   (register or immediate mode)
    CMP Rn, Rm|#imm
    B label | B_<cond> label   (cond: EQ NE CS HS CC LO MI PL VS VC HI LS GE LT GT LE AL)
    HALT

Labels end with ':'. Comments start with ';' or '//'. Commas are optional.
MUL returns the low W bits of the paper's sequential multiplier. UDIV is
the non-restoring divider.
"""
from __future__ import annotations

import re
from dataclasses import dataclass

import numpy as np

from . import cemu
from . import circuits as C

ALU_KINDS = {
    "ADD": "ADD", "SUB": "SUB", "MUL": "MULSEQ", "UDIV": "DIV", "AND": "AND", "ORR": "OR", "EOR": "XOR",
    "ORN": "ORN", "LSL": C.LLS, "LLS": C.LLS, "LSR": C.LRS, "LRS": C.LRS, "ASR": C.ARS, "ARS": C.ARS,
}
FLAG_KINDS = {"ADDS": "ADDS", "SUBS": "SUBS", "CMP": "CMP"}
SHIFTS = (C.LLS, C.LRS, C.ARS)
CONDS = ("EQ", "NE", "CS", "HS", "CC", "LO", "MI", "PL", "VS", "VC", "HI", "LS", "GE", "LT", "GT", "LE", "AL")


@dataclass
class Instr:
    op: str
    rd: int = -1
    rn: int = -1
    rm: int = -1            # register operand, or -1
    imm: int | None = None  # immediate operand
    target: str = ""        # branch label
    cond: str = "AL"
    text: str = ""


def _reg(tok: str) -> int:
    m = re.fullmatch(r"[Rr](\d+)", tok)
    if not m:
        raise ValueError(f"expected a register, got {tok!r}")
    return int(m.group(1))


def _imm(tok: str) -> int:
    return int(tok.lstrip("#"), 0)


def _is_reg(tok: str) -> bool:
    return re.fullmatch(r"[Rr]\d+", tok) is not None


def assemble(text: str):
    """Parse assembly into (instructions, {label: index})."""
    prog, labels = [], {}
    for raw in text.splitlines():
        line = re.split(r";|//", raw, maxsplit=1)[0].strip()
        if not line:
            continue
        while ":" in line:
            lab, line = line.split(":", 1)
            labels[lab.strip()] = len(prog)
            line = line.strip()
        if not line:
            continue
        toks = line.replace(",", " ").split()
        op, args = toks[0].upper(), toks[1:]
        if op == "HALT":
            prog.append(Instr("HALT", text=line))
        elif op == "B" or op.startswith("B_"):
            cond = "AL" if op == "B" else op[2:]
            if cond not in CONDS:
                raise ValueError(f"unknown branch condition in {line!r}")
            prog.append(Instr("B", target=args[0], cond=cond, text=line))
        elif op in ("LOAD", "STORE"):
            prog.append(Instr(op, rd=_reg(args[0]), imm=_imm(args[1]), text=line))
        elif op == "MOV":
            if len(args) == 3:          # MOV Rd, Rn, #imm (the paper's form)
                prog.append(Instr("MOV", rd=_reg(args[0]), imm=_imm(args[2]), text=line))
            elif _is_reg(args[1]):
                prog.append(Instr("MOV", rd=_reg(args[0]), rm=_reg(args[1]), text=line))
            else:
                prog.append(Instr("MOV", rd=_reg(args[0]), imm=_imm(args[1]), text=line))
        elif op == "MVN":
            prog.append(Instr("MVN", rd=_reg(args[0]), rm=_reg(args[1]), text=line))
        elif op == "CMP":
            ins = Instr("CMP", rn=_reg(args[0]), text=line)
            if _is_reg(args[1]):
                ins.rm = _reg(args[1])
            else:
                ins.imm = _imm(args[1])
            prog.append(ins)
        elif op in ALU_KINDS or op in FLAG_KINDS:
            ins = Instr(op, rd=_reg(args[0]), rn=_reg(args[1]), text=line)
            if _is_reg(args[2]):
                ins.rm = _reg(args[2])
            else:
                ins.imm = _imm(args[2])
            prog.append(ins)
        else:
            raise ValueError(f"unknown instruction {op!r}")
    for ins in prog:
        if ins.op == "B" and ins.target not in labels:
            raise ValueError(f"undefined label {ins.target!r}")
    return prog, labels


def condition_holds(cond: str, n: int, z: int, c: int, v: int) -> bool:
    """ARM condition codes on cleartext flags."""
    return {
        "EQ": z == 1, "NE": z == 0, "CS": c == 1, "HS": c == 1, "CC": c == 0, "LO": c == 0,
        "MI": n == 1, "PL": n == 0, "VS": v == 1, "VC": v == 0, "HI": c == 1 and z == 0,
        "LS": c == 0 or z == 1, "GE": n == v, "LT": n != v, "GT": z == 0 and n == v,
        "LE": z == 1 or n != v, "AL": True,
    }[cond]


def make_client(keys: cemu.Keys):
    """The user's side of branch resolution: decrypt the flags with the secret
    key and answer taken / not taken. Returns callback(cond, nzcv_ct) where
    nzcv_ct is the host copy [4][n+1] of the encrypted N, Z, C, V."""
    def client(cond: str, nzcv_ct: np.ndarray) -> bool:
        n, z, c, v = (int(x) for x in keys.decrypt(nzcv_ct))
        return condition_holds(cond, n, z, c, v)
    return client


class _Unit:
    """One data-processing circuit with its own ciphertext pool: inputs a, b
    (W rows each) and outputs 'out' (and 'nzcv')."""

    def __init__(self, circuit: C.Circuit, keys, device):
        import torch
        self.circuit = circuit
        self.program = C.Program([circuit]).to_device(device)
        self.pool = torch.zeros((self.program.rows, keys.n + 1), dtype=torch.int32, device=device)
        W = len(circuit.inputs) // 2

        def t(a):
            return torch.as_tensor(np.asarray(a, np.int32), device=device)
        self.in_a = t(circuit.inputs[:W])
        self.in_b = t(circuit.inputs[W:])
        self.out = t(circuit.outputs["out"])
        self.nzcv = t(circuit.outputs["nzcv"]) if "nzcv" in circuit.outputs else None


class Machine:
    """Emulator state on one GPU: registers [nregs][W] and HE data memory
    [mem_words][W] as ciphertext pools, NZCV as a 4-row pool, a cleartext PC.

    form / tuner: the product form and the autotuner (or ``None`` for the
    form with the cloud key's current launch shape) used by every level.
    prefix: the adders' prefix form (circuits.PREFIX_GATES, the paper's, or
    circuits.PREFIX_MUX, fewer levels)."""

    def __init__(self, keys: cemu.Keys, width: int = 32, nregs: int = 16, mem_words: int = 0, form: str = "fft64",
                 tuner=None, device=None, prefix: str = C.PREFIX_GATES):
        import torch
        self.keys, self.W, self.form, self.tuner, self.prefix = keys, width, form, tuner, prefix
        self.device = device if device is not None else torch.device("cuda", torch.cuda.current_device())
        n1 = keys.n + 1
        self.regs = torch.zeros((nregs * width, n1), dtype=torch.int32, device=self.device)
        self.mem = torch.zeros((max(mem_words, 1) * width, n1), dtype=torch.int32, device=self.device)
        self.flags = torch.zeros((4, n1), dtype=torch.int32, device=self.device)
        self.nregs, self.mem_words = nregs, mem_words
        self._units = {}
        self._rows = torch.arange(max(nregs, mem_words, 1) * width, dtype=torch.int32, device=self.device)
        zero = torch.zeros(4, dtype=torch.uint8, device=self.device)
        cemu.lwe_constant(keys.n, zero, self.flags, self._rows[:4])
        self.pc = 0
        self.stats = {"instructions": 0, "branches": 0, "bootstraps": 0, "levels": 0}

    # ------------------------------------------------------------ host I/O
    def _reg_rows(self, r: int):
        if not 0 <= r < self.nregs:
            raise ValueError(f"register R{r} out of range")
        return self._rows[r * self.W:(r + 1) * self.W]

    def _mem_rows(self, a: int):
        if not 0 <= a < self.mem_words:
            raise ValueError(f"memory word {a} out of range")
        return self._rows[a * self.W:(a + 1) * self.W]

    def write_memory(self, ct: np.ndarray):
        """ct: host uint32 [words][W][n+1] ciphertexts (the user's encrypted data)."""
        import torch
        ct = np.ascontiguousarray(ct, dtype=np.uint32).reshape(-1, self.keys.n + 1)
        self.mem[:ct.shape[0]] = torch.from_numpy(ct.view(np.int32)).to(self.device)

    def read_memory(self) -> np.ndarray:
        return self.mem.cpu().numpy().view(np.uint32).reshape(-1, self.W, self.keys.n + 1)[:self.mem_words]

    def read_register(self, r: int) -> np.ndarray:
        rows = self._reg_rows(r).long()
        return self.regs[rows].cpu().numpy().view(np.uint32)

    def read_flags(self) -> np.ndarray:
        return self.flags.cpu().numpy().view(np.uint32)

    # ------------------------------------------------------------ execution
    def _unit(self, kind: str, imm_shift: int | None = None) -> _Unit:
        key = (kind, imm_shift)
        if key not in self._units:
            if kind in FLAG_KINDS.values():
                circ = C.flag_setting_circuit(kind, self.W, self.prefix)
            elif imm_shift is not None:
                circ = C.Circuit()
                A = circ.inputs_word(self.W)
                circ.inputs_word(self.W)               # unused second operand keeps the layout uniform
                circ.outputs["out"] = C.shift_immediate(circ, A, imm_shift, kind)
            else:
                circ = C.instruction_circuit(kind, self.W, self.prefix)
            self._units[key] = _Unit(circ, self.keys, self.device)
        return self._units[key]

    def _constant_into(self, value: int, pool, rows):
        import torch
        bits = torch.as_tensor(np.array(C.int_to_bits(value & ((1 << self.W) - 1), self.W), np.uint8),
                               device=self.device)
        cemu.lwe_constant(self.keys.n, bits, pool, rows)

    def _alu(self, ins: Instr, kind: str):
        n = self.keys.n
        shift_imm = ins.imm if (kind in SHIFTS and ins.imm is not None) else None
        u = self._unit(kind, shift_imm)
        cemu.lwe_copy(n, self.regs, self._reg_rows(ins.rn), u.pool, u.in_a)
        if shift_imm is None:
            if ins.rm >= 0:
                cemu.lwe_copy(n, self.regs, self._reg_rows(ins.rm), u.pool, u.in_b)
            else:
                self._constant_into(ins.imm, u.pool, u.in_b)
        u.program.run(self.keys, u.pool, form=self.form, tuner=self.tuner)
        W = self.W
        if ins.op != "CMP":
            out = u.out[:W] if kind == "MULSEQ" else u.out
            cemu.lwe_copy(n, u.pool, out, self.regs, self._reg_rows(ins.rd))
        if u.nzcv is not None:
            cemu.lwe_copy(n, u.pool, u.nzcv, self.flags, self._rows[:4])
        self.stats["bootstraps"] += u.program.num_bootstraps()
        self.stats["levels"] += u.program.depth

    def step(self, prog, labels, client) -> bool:
        """Execute the instruction at the PC; False once the program halts."""
        if not 0 <= self.pc < len(prog):
            return False
        ins = prog[self.pc]
        n = self.keys.n
        nxt = self.pc + 1
        if ins.op == "HALT":
            return False
        if ins.op == "MOV":
            if ins.rm >= 0:
                cemu.lwe_copy(n, self.regs, self._reg_rows(ins.rm), self.regs, self._reg_rows(ins.rd))
            else:
                self._constant_into(ins.imm, self.regs, self._reg_rows(ins.rd))
        elif ins.op == "MVN":
            cemu.lwe_not(n, self.regs, self._reg_rows(ins.rm), self.regs, self._reg_rows(ins.rd))
        elif ins.op == "LOAD":
            cemu.lwe_copy(n, self.mem, self._mem_rows(ins.imm), self.regs, self._reg_rows(ins.rd))
        elif ins.op == "STORE":
            cemu.lwe_copy(n, self.regs, self._reg_rows(ins.rd), self.mem, self._mem_rows(ins.imm))
        elif ins.op == "B":
            self.stats["branches"] += 1
            taken = True if ins.cond == "AL" else bool(client(ins.cond, self.read_flags()))
            if taken:
                nxt = labels[ins.target]
        elif ins.op in FLAG_KINDS:
            self._alu(ins, FLAG_KINDS[ins.op])
        else:
            self._alu(ins, ALU_KINDS[ins.op])
        self.stats["instructions"] += 1
        self.pc = nxt
        return True

    def run(self, program, client=None, max_steps: int = 100000) -> dict:
        """Run assembly text (or an assembled (prog, labels) pair) from PC 0
        until HALT, the end of the program or max_steps instructions.
        client: branch-resolution callback (see make_client); needed only for
        conditional branches."""
        prog, labels = assemble(program) if isinstance(program, str) else program
        self.pc = 0
        for _ in range(max_steps):
            if not self.step(prog, labels, client):
                break
        else:
            raise RuntimeError(f"program did not halt within {max_steps} instructions")
        return dict(self.stats, pc_bytes=4 * self.pc)
