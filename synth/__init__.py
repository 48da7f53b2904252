"""Seeded synthetic gate-stack devices: the inputs both the solver and its checker consume.

This package only lays out meshes, materials, doping, gate rectangles and
contact voltages.  It holds none of the solver's arithmetic (no charge
statistics, no discretisation, no physical constants).
"""
from .devices import (  # noqa: F401
    doped_block,
    with_species,
    with_interface_charge,
    with_charged_gates,
    Sheet,
    QuantumStates,
    box_states,
    with_quantum,
    quantum_region,
    Device,
    stack_z,
    make_stack_device,
    double_dot_gates,
    PLUNGER_GRID,
    double_dot_device,
    config1,
    config2,
    config3_spec,
    config3_instance,
    config4,
    config5,
    DOT_BOX_D1,
    DOT_BOX_D2,
)
