"""The host-side checks of the C ABI (test_abi.py: every declared symbol is
exported, workspace sizes, status strings, argument validation before any
launch), run again in the GPU session, so that they are recorded there too."""
import pytest

from test_abi import (test_header_declares_the_three_calls,  # noqa: F401
                      test_invalid_arguments_rejected_before_launch,
                      test_library_exports_every_declared_symbol, test_sinkhorn_and_solve_validation,
                      test_status_strings, test_workspace_bytes_arithmetic)

pytestmark = pytest.mark.gpu
