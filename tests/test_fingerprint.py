"""The kernels' assembly fingerprints that tie a counter summary to the code
it measured: the parser keeps instructions and labels of each kernel and
drops comments, line records and directives, so a fingerprint changes with
the code and with nothing else."""
import hashlib

from paper_2401_04701_amd import build as hb

LISTING = """\t.text
\t.globl\tk_a
\t.type\tk_a,@function
k_a:                                    ; @k_a
\t.loc\t1 10 0
\ts_load_dword s0, s[0:1], 0x0 ; a comment
.LBB0_1:
\tv_add_u32_e32 v0, s0, v0
\ts_endpgm
.Lfunc_end0:
\t.size\tk_a, .Lfunc_end0-k_a
\t.globl\thelper
helper:
\ts_setpc_b64 s[30:31]
.Lfunc_end1:
\t.amdhsa_kernel k_a
\t.end_amdhsa_kernel
"""


def test_parser_keeps_code_only():
    bodies = hb._kernel_bodies(LISTING)
    assert list(bodies) == ["k_a"]                       # helper is not a kernel
    assert bodies["k_a"].splitlines() == ["s_load_dword s0, s[0:1], 0x0", ".LBB_1:",
                                          "v_add_u32_e32 v0, s0, v0", "s_endpgm"]


def test_fingerprint_ignores_label_function_numbers():
    """Adding a function before a kernel renumbers its local labels only."""
    a = hb._kernel_bodies(LISTING)["k_a"]
    b = hb._kernel_bodies(LISTING.replace(".LBB0_1", ".LBB7_1"))["k_a"]
    c = hb._kernel_bodies(LISTING.replace(".LBB0_1", ".LBB0_2"))["k_a"]
    assert a == b and a != c


def test_fingerprint_ignores_comments_and_line_records():
    a = hb._kernel_bodies(LISTING)["k_a"]
    b = hb._kernel_bodies(LISTING.replace("; a comment", "; other").replace(
        "\t.loc\t1 10 0", "\t.loc\t2 99 3"))["k_a"]
    c = hb._kernel_bodies(LISTING.replace("v_add_u32_e32", "v_sub_u32_e32"))["k_a"]
    h = [hashlib.sha256(x.encode()).hexdigest() for x in (a, b, c)]
    assert h[0] == h[1] and h[0] != h[2]
